"""Batched form (many datasets per launch) against stored FP64 oracle runs.

Raw data in, unique sets out, through ordering_ica_batched (batched whitening,
one batched fixed point, batched unique) in both forms: BF16 data with the
grouped FP32 finish (the form the benchmark times) and plain FP32.  Each side
whitens by itself, so components are compared in raw-data space.

* batched_basins: one dataset per padded-dimension class (N = 20, 40, 80, 110;
  the BF16 kernel variants for 32, 64, 96 and 128 features), T = 2e4, with
  1024 to 6144 starts.
* batched_n16_128: the 64-dataset workload as benchmarked (N uniform over
  {16, ..., 128}, T log-uniform in [2e4, 5e5], K = 1024 each), all 64 in one
  call; checked against the oracle on the two datasets with the smallest N T
  of each class (eight datasets), and every dataset's BF16 set against its
  FP32 set.

Oracle runs: tests/golden/batched_basins_oracle.json and
batched_n16_128_oracle.json, written by tests/golden/make_reference.py (calls
only the generator and oracle/).

Contract per dataset (reading of rare basins): every oracle cluster is found,
one to one, at |cos| >= 1 - 1e-6 with kurtosis within 1e-5 max(|alpha|, 0.1),
whatever its size (single-start clusters included); in the same order up to
groups of near-equal criterion values.  The GPU run may hold extra clusters
only of at most two starts -- a start near a basin boundary can settle at
another fixed point under another rounding -- and its accepted count may
exceed the oracle's by those alone.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2408_17118_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden")
sys.path.insert(0, GOLD)
import make_reference as mr  # noqa: E402  (shapes and the dataset selection only)


def compare_with_oracle(res, ref, label):
    ng, nu = res["n_accepted"], res["n_unique"]
    U = res["U"].cpu().numpy()[:nu] @ res["V"].cpu().numpy()
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    Ur = np.asarray(ref["U_raw"])
    cos = np.abs(U @ Ur.T) if nu and len(Ur) else np.zeros((nu, len(Ur)))
    sg = res["size"].cpu().numpy()[:nu]
    a = res["alpha"].cpu().numpy()[:nu]
    ar, upr = np.asarray(ref["alpha"]), np.asarray(ref["upsilon"])
    # every oracle cluster found, one to one
    best_g = cos.argmax(axis=0)
    assert np.all(cos.max(axis=0) >= 1 - 1e-6), (label, np.flatnonzero(cos.max(axis=0) < 1 - 1e-6))
    assert len(set(best_g.tolist())) == len(Ur), label
    # extra GPU clusters: at most two starts each
    extra = np.setdiff1d(np.arange(nu), best_g)
    assert np.all(sg[extra] <= 2), (label, extra, sg[extra])
    extra_acc = int(np.sum(extra < ng))
    assert ng == ref["n_accepted"] + extra_acc, (label, ng, ref["n_accepted"], extra_acc)
    # kurtosis and order of the matched clusters
    rel = np.abs(a[best_g] - ar) / np.maximum(np.abs(ar), 0.1)
    assert np.all(rel <= 1e-5), (label, rel.max())
    matched = [i for i in range(nu) if i not in set(extra.tolist())]
    order = [int(cos[i].argmax()) for i in matched]
    for k, j in enumerate(order):
        if j != k:
            assert abs(upr[j] - upr[k]) <= 1e-5 * max(upr[k], 1e-3), (label, k, j)
    return len(extra)


def _run(ctx, Xs, W0s, precision):
    from paper_2408_17118_amd import oica
    res, st = oica.ordering_ica_batched(ctx, Xs, W0s, tol=1e-6, max_iter=1000, precision=precision,
                                        refine_iters=5)
    return res


@pytest.fixture(scope="module")
def ctx():
    from paper_2408_17118_amd import oica
    c = oica.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("precision", ["bf16", "f32"])
def test_one_dataset_per_class_matches_oracle(ctx, precision):
    gold = json.load(open(os.path.join(GOLD, "batched_basins_oracle.json")))["datasets"]
    probs = [synth.make_problem(synth.eeg_kinds(N), T=T, K=K, seed=seed)
             for N, T, K, seed in mr.BASIN_SHAPES]
    Xs = [torch.from_numpy(p.X).cuda() for p in probs]
    W0s = [torch.from_numpy(p.W0.astype(np.float32)).cuda() for p in probs]
    res = _run(ctx, Xs, W0s, precision)
    for e in gold:
        d = e["dataset"]
        n_extra = compare_with_oracle(res[d], e, f"{precision} N={e['N']} K={e['K']}")
        print(f"{precision} N={e['N']} K={e['K']}: {res[d]['n_accepted']} accepted "
              f"(oracle {e['n_accepted']}), extra small clusters {n_extra}")


@pytest.fixture(scope="module")
def full_batch(ctx):
    shapes = synth.batched_shapes()
    Xs, W0s = [], []
    for N, T, rng in shapes:
        p = synth.batched_problem(N, T, rng)
        Xs.append(torch.from_numpy(p.X).cuda())
        W0s.append(torch.from_numpy(p.W0.astype(np.float32)).cuda())
        del p
    out = {prec: _run(ctx, Xs, W0s, prec) for prec in ("bf16", "f32")}
    del Xs
    torch.cuda.empty_cache()
    return shapes, out


@pytest.mark.slow
@pytest.mark.parametrize("precision", ["bf16", "f32"])
def test_full_workload_matches_oracle(full_batch, precision):
    shapes, out = full_batch
    gold = json.load(open(os.path.join(GOLD, "batched_n16_128_oracle.json")))["datasets"]
    assert [e["dataset"] for e in gold] == mr.batched_selection(shapes)
    classes = set()
    for e in gold:
        d = e["dataset"]
        n_extra = compare_with_oracle(out[precision][d], e, f"{precision} dataset {d}")
        classes.add((e["N"] + 31) // 32 * 32)
        print(f"{precision} dataset {d} N={e['N']} T={e['T']}: {out[precision][d]['n_accepted']} "
              f"accepted (oracle {e['n_accepted']}), extra small clusters {n_extra}")
    assert classes == {32, 64, 96, 128}


@pytest.mark.slow
def test_full_workload_bf16_matches_f32(full_batch):
    """Every dataset: the BF16 set against the FP32 set (the FP32 run standing in
    for the oracle on the 56 datasets without a stored oracle run): a cluster
    found by one form only may hold at most two starts; the others match at
    |cos| >= 1 - 1e-6 with kurtosis within 1e-5 max(|alpha|, 0.1)."""
    shapes, out = full_batch
    extras = 0
    for d in range(len(shapes)):
        extras += _compare_two(out["bf16"][d], out["f32"][d], f"dataset {d}")
    print(f"clusters of <= 2 starts found by one form only: {extras}")


def _raw_set(res):
    nu = res["n_unique"]
    U = res["U"].cpu().numpy()[:nu] @ res["V"].cpu().numpy()
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    return U, res["alpha"].cpu().numpy()[:nu], res["size"].cpu().numpy()[:nu]


def _compare_two(ra, rb, label):
    Ua, aa, sa = _raw_set(ra)
    Ub, ab, sb = _raw_set(rb)
    cos = np.abs(Ua @ Ub.T)
    only = 0
    for X_cos, s_x, a_x, a_y in ((cos, sa, aa, ab), (cos.T, sb, ab, aa)):
        for i in range(len(s_x)):
            j = int(X_cos[i].argmax()) if X_cos.shape[1] else -1
            if j >= 0 and X_cos[i, j] >= 1 - 1e-6:
                assert abs(a_x[i] - a_y[j]) <= 1e-5 * max(abs(a_y[j]), 0.1), (label, i)
            else:
                assert s_x[i] <= 2, (label, i, int(s_x[i]))
                only += 1
    return only
