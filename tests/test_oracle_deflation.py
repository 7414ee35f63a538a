"""Pins of the oracle's deflation driver (Algorithm 2's outer loop, Sec. 3.3,
eqs. 6-8) against routes that do not share its arithmetic:

* the reduced basis G = (F~ F~^T)^(-1/2) F~ equals the polar factor U V^T of
  F~'s singular value decomposition (another LAPACK route), has orthonormal
  rows, and is orthogonal to the components found so far;
* a step's fixed point on the reduced data X~ = G Xw, mapped back by G, is
  Algorithm 1's FastICA with the projection E = W^T W run in the full space
  (no reduction, no inverse square root);
* the components are orthonormal and recover the known mixing matrix in the
  order of the sources' criterion values, with the Gaussianity break of eq. 3
  where the planted Gaussian sources begin;
* planted mistakes (no orthonormalisation of F~, the reduced row appended
  without mapping it back) fail these pins.
"""
import numpy as np
import pytest

from oracle import ica
from paper_2408_17118_amd import synth


@pytest.fixture(scope="module")
def small():
    p = synth.small_mixture()
    Xw, V, mu, lam = ica.whiten(p.X)
    W0s = synth.draw_deflation_starts(np.random.default_rng(10), 256, p.N)
    W, steps = ica.deflation(Xw, W0s, 1e-10, 1000)
    return p, Xw, V, W0s, W, steps


def check_basis(W, N):
    G = ica.reduce_basis(W, N)
    n = N - W.shape[0]
    assert G.shape == (n, N)
    assert np.max(np.abs(G @ G.T - np.eye(n))) < 1e-12
    if W.shape[0]:
        assert np.max(np.abs(W @ G.T)) < 1e-12
        Ft = (np.eye(N) - W.T @ W)[:n]
        U, s, Vt = np.linalg.svd(Ft, full_matrices=False)
        assert np.max(np.abs(G - U @ Vt)) < 1e-10
    return G


def test_reduced_basis(small):
    p, Xw, V, W0s, W, steps = small
    assert np.array_equal(ica.reduce_basis(np.zeros((0, p.N)), p.N), np.eye(p.N))
    for k in range(W.shape[0]):
        check_basis(W[:k], p.N)


def test_components_orthonormal(small):
    p, Xw, V, W0s, W, steps = small
    assert np.max(np.abs(W @ W.T - np.eye(W.shape[0]))) < 1e-12


def test_orthonormal_over_many_steps():
    # sixteen steps on the EEG-shaped family mix: the components stay
    # orthonormal to FP64 rounding (the appended rows are re-orthogonalised),
    # and every step's basis is orthonormal and orthogonal to them
    p = synth.make_problem(synth.eeg_kinds(16), T=20_000, K=4, seed=12)
    Xw, *_ = ica.whiten(p.X)
    W0s = synth.draw_deflation_starts(np.random.default_rng(13), 128, p.N)
    W, steps = ica.deflation(Xw, W0s, 1e-10, 1000, gaussianity_test=False)
    assert W.shape == (16, 16) and len(steps) == 16
    assert np.max(np.abs(W @ W.T - np.eye(16))) < 1e-13
    for k in range(1, 16):
        G = ica.reduce_basis(W[:k], 16)
        assert np.max(np.abs(W[:k] @ G.T)) < 1e-11
        assert np.max(np.abs(G @ G.T - np.eye(16 - k))) < 1e-8


def test_step_equals_projected_fastica(small):
    # step 3: the reduced fixed point mapped back equals Algorithm 1's
    # projected FastICA from the same start, row by row
    p, Xw, V, W0s, W, steps = small
    Wp = W[:2]
    G = ica.reduce_basis(Wp, p.N)
    rows = W0s[2][:12]
    B, iters, status, _, _ = ica.fixed_point(G @ Xw, rows, 1e-10, 1000)
    E = Wp.T @ Wp
    for l in range(rows.shape[0]):
        w, t, conv = ica.fastica_projected(Xw, rows[l] @ G, E, 1e-10, 1000)
        assert conv and status[l] == ica.CONV
        assert t == iters[l]
        assert np.max(np.abs(w - B[l] @ G)) < 1e-11


def test_first_step_is_the_plain_argmax(small):
    p, Xw, V, W0s, W, steps = small
    B, it, st, _, _ = ica.fixed_point(Xw, W0s[0], 1e-10, 1000)
    res = ica.unique(B, ica.kurtosis(Xw, B), st, p.T, n_top=1)
    assert steps[0]["p"] == res["rep"][0]
    assert abs(abs(float(W[0] @ B[res["rep"][0]])) - 1) < 1e-14


def test_recovery_in_criterion_order(small):
    p, Xw, V, W0s, W, steps = small
    ng = [j for j, k in enumerate(p.kinds) if k != "gaussian"]
    C = (W[: len(ng)] @ V) @ p.A          # rows ~ +-e_j
    purity = np.max(np.abs(C), axis=1) / np.linalg.norm(C, axis=1)
    assert np.all(purity >= 0.99)
    matched = list(np.argmax(np.abs(C), axis=1))
    assert sorted(matched) == ng
    S = p.S - p.S.mean(axis=1, keepdims=True)
    kap = (S ** 4).mean(axis=1) / (S ** 2).mean(axis=1) ** 2 - 3
    assert matched == sorted(ng, key=lambda j: -ica.upsilon(kap[j]))
    for s in steps:
        assert s["accepted"] == (s["upsilon"] >= s["threshold"])
        assert s["threshold"] == pytest.approx(2 * (p.N - s["i"] + 2) * (p.N - s["i"] + 1) / p.T)


def test_gaussianity_break():
    # three Laplace and three Gaussian sources: the three Laplace sources, then
    # the first step whose criterion falls below eq. 3's threshold ends the loop
    p = synth.make_problem(["laplace"] * 3 + ["gaussian"] * 3, T=100_000, K=64, seed=3)
    Xw, V, mu, lam = ica.whiten(p.X)
    W0s = synth.draw_deflation_starts(np.random.default_rng(53), 64, p.N)
    W, steps = ica.deflation(Xw, W0s, 1e-10, 1000)
    assert W.shape[0] == 3 and len(steps) == 4 and not steps[-1]["accepted"]
    C = (W @ V) @ p.A
    assert sorted(np.argmax(np.abs(C), axis=1)) == [0, 1, 2]


def test_rank_error():
    # F~ F~^T singular: a found component lying in the span of the first
    # N - i + 1 coordinates leaves the first rows of F dependent
    W = np.array([[1.0, 0.0, 0.0]])
    with pytest.raises(ica.RankError):
        ica.reduce_basis(W, 3)


_reduce = ica.reduce_basis


def test_mutation_no_orthonormalisation_caught(monkeypatch, small):
    p, Xw, V, W0s, W, steps = small

    def rb(W, N, rank_tol=1e-12):
        W = np.asarray(W, dtype=np.float64).reshape(-1, N)
        if W.shape[0] == 0:
            return np.eye(N)
        return (np.eye(N) - W.T @ W)[: N - W.shape[0]]
    monkeypatch.setattr(ica, "reduce_basis", rb)
    with pytest.raises(AssertionError):
        check_basis(W[:2], p.N)


def test_mutation_reduced_row_not_mapped_back_caught(monkeypatch):
    p = synth.small_mixture()
    Xw, V, mu, lam = ica.whiten(p.X)
    W0s = synth.draw_deflation_starts(np.random.default_rng(10), 64, p.N)

    def defl(Xw, W0s, tol, max_iter, rank_tol=1e-12):
        N, T = Xw.shape
        W = np.zeros((0, N))
        for i in range(1, N + 1):
            G = _reduce(W, N)
            Xt = G @ Xw
            B, it, st, _, _ = ica.fixed_point(Xt, W0s[i - 1], tol, max_iter)
            ups = ica.upsilon(ica.kurtosis(Xt, B))
            p_ = int(np.argmax(ups))
            row = np.zeros(N)
            row[: N - i + 1] = B[p_]          # mistake: b_p instead of b_p G
            W = np.vstack([W, row])
        return W, []
    W, _ = defl(Xw, W0s, 1e-10, 1000)
    with pytest.raises(AssertionError):
        assert np.max(np.abs(W @ W.T - np.eye(W.shape[0]))) < 1e-12


# ---- Algorithm 1 (the original ordering ICA) ----------------------------------

def test_original_algorithm_first_step_is_plain_fastica(small):
    p, Xw, V, W0s, W, steps = small
    starts = synth.draw_original_starts(np.random.default_rng(21), 16, p.N)
    for l in range(4):
        w1, t1, c1 = ica.fastica_projected(Xw, starts[0][l], np.zeros((p.N, p.N)), 1e-10, 1000)
        w2, t2, c2 = ica.fastica_single(Xw, starts[0][l], 1e-10, 1000)
        assert t1 == t2 and c1 == c2 and np.max(np.abs(w1 - w2)) < 1e-15


def test_original_algorithm_recovers_sources(small):
    # Algorithm 1 on the small mixture: orthonormal components, the known
    # sources in criterion order, the same components as the fast form
    p, Xw, V, W0s, W_fast, steps_fast = small
    starts = synth.draw_original_starts(np.random.default_rng(22), 64, p.N)
    W, steps = ica.ordering_original(Xw, starts, 1e-10, 1000)
    assert np.max(np.abs(W @ W.T - np.eye(len(W)))) < 1e-12
    ng = [j for j, k in enumerate(p.kinds) if k != "gaussian"]
    C = (W[: len(ng)] @ V) @ p.A
    assert np.all(np.max(np.abs(C), axis=1) / np.linalg.norm(C, axis=1) >= 0.99)
    assert sorted(np.argmax(np.abs(C), axis=1)) == ng
    n = min(len(W), len(W_fast))
    assert np.all(np.abs(np.einsum("kn,kn->k", W[:n], W_fast[:n])) >= 1 - 1e-6)
    for s in steps:
        assert s["accepted"] == (s["upsilon"] >= s["threshold"])
