"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin fails.

Each mutation replaces one oracle function for the duration of a test; the pin
functions of ``test_oracle_pins`` are then called and must raise.  This shows
that the pins would have caught the mistake.
"""
import numpy as np
import pytest

import test_oracle_pins as pins
from oracle import ica
from paper_2408_17118_amd import synth

_update = ica.update
_whiten = ica.whiten


def _small():
    p = synth.small_mixture()
    Xw, V, mu, lam = _whiten(p.X)
    return p, Xw, V, mu, lam


def _mut_update(kind):
    def upd(Xw, P):
        N, T = Xw.shape
        G = np.zeros_like(P)
        s4 = np.zeros(P.shape[0])
        Z = P @ Xw
        if kind == "drop_minus_3b":
            return (Z ** 3) @ Xw.T / T, (Z ** 4).sum(1) / T
        if kind == "plus_3b":
            return (Z ** 3) @ Xw.T / T + 3 * P, (Z ** 4).sum(1) / T
        if kind == "square":
            return (Z ** 2) @ Xw.T / T - 3 * P, (Z ** 4).sum(1) / T
        if kind == "minus_1b":
            return (Z ** 3) @ Xw.T / T - 1 * P, (Z ** 4).sum(1) / T
        if kind == "unscaled":
            return (Z ** 3) @ Xw.T - 3 * P, (Z ** 4).sum(1) / T
        raise ValueError(kind)
    return upd


@pytest.mark.parametrize("kind", ["drop_minus_3b", "plus_3b", "square", "minus_1b", "unscaled"])
def test_update_mutations_caught(monkeypatch, kind):
    monkeypatch.setattr(ica, "update", _mut_update(kind))
    caught = 0
    for pin in (pins.test_update_identity, pins.test_fixed_point_limits):
        try:
            pin(_small())
        except (AssertionError, FloatingPointError, ValueError):
            caught += 1
    # the matrix form must also disagree with the library FastICA
    try:
        pins.test_update_matches_library_fastica(_small())
    except AssertionError:
        caught += 1
    assert caught >= 1


@pytest.mark.parametrize("kind", ["t_minus_1", "no_sign_fix", "no_centre"])
def test_whiten_mutations_caught(monkeypatch, kind):
    def wh(X, rank_tol=1e-12):
        X = np.asarray(X, dtype=np.float64)
        N, T = X.shape
        mu = X.mean(axis=1)
        Xc = X - mu[:, None] if kind != "no_centre" else X.copy()
        C = Xc @ Xc.T / (T - 1 if kind == "t_minus_1" else T)
        lam, E = np.linalg.eigh(C)
        o = np.argsort(-lam, kind="stable")
        lam, E = lam[o], E[:, o]
        if kind != "no_sign_fix":
            for j in range(N):
                if E[np.argmax(np.abs(E[:, j])), j] < 0:
                    E[:, j] = -E[:, j]
        else:
            E = -E
        V = (E / np.sqrt(lam)).T
        return V @ Xc, V, mu, lam
    monkeypatch.setattr(ica, "whiten", wh)
    p = synth.make_problem(["laplace"] * 4 + ["uniform"] * 4, T=10_000, K=8, seed=3)
    p.X += 0.7   # non-zero means, so a missing centring step shows
    Xw, V, mu, lam = ica.whiten(p.X)
    with pytest.raises(AssertionError):
        pins.test_whiten_identity_covariance((p, Xw, V, mu, lam))


def test_unique_sign_sensitive_mutation_caught(monkeypatch):
    # cluster on cos instead of |cos|: copies of one component with opposite
    # signs fall into separate clusters
    monkeypatch.setattr(ica, "unique", lambda B, alpha, status, T, tau=1e-3, gaussianity_test=True,
                        n_top=0: _greedy_signed(B, alpha, status, tau))
    with pytest.raises(AssertionError):
        pins.test_unique_planted_clusters()


def _greedy_signed(B, alpha, status, tau):
    # same as the oracle but with the sign-sensitive distance 1 - b.b_r
    ups = ica.upsilon(alpha)
    cand = np.flatnonzero(status == ica.CONV)
    order = cand[np.lexsort((cand, -ups[cand]))]
    reps, sizes = [], []
    for l in order:
        for j, r in enumerate(reps):
            if 1.0 - float(B[l] @ B[r]) <= tau:
                sizes[j] += 1
                break
        else:
            reps.append(l)
            sizes.append(1)
    return {"U": np.array([ica.canonical_sign(B[r]) for r in reps]), "alpha": alpha[reps],
            "upsilon": ups[reps], "rep": np.array(reps), "size": np.array(sizes),
            "n_accepted": len(reps)}


def test_s4_from_updated_rows_caught(monkeypatch):
    # the kurtosis by-product taken from the normalised new rows instead of the
    # rows the pass started from
    def upd(Xw, P):
        G, _ = _update(Xw, P)
        Bn = G / np.linalg.norm(G, axis=1, keepdims=True)
        _, s4n = _update(Xw, Bn)
        return G, s4n
    monkeypatch.setattr(ica, "update", upd)
    with pytest.raises(AssertionError):
        pins.test_update_s4_matches_scipy(_small())


_fixed_point = ica.fixed_point


@pytest.mark.parametrize("kind", ["shift_one_pass", "alpha_after_update"])
def test_trajectory_mutations_caught(monkeypatch, kind):
    def fp(Xw, W0, tol, max_iter, traj_iters=0):
        B, iters, status, traj, ti = _fixed_point(Xw, W0, tol, max_iter, traj_iters)
        traj = traj.copy()
        if kind == "shift_one_pass":        # record of pass t stored at t + 1
            traj[:, 1:] = traj[:, :-1].copy()
        else:                               # kurtosis of the row after the pass
            traj[:, :-1, 0] = traj[:, 1:, 0].copy()
        return B, iters, status, traj, ti
    monkeypatch.setattr(ica, "fixed_point", fp)
    with pytest.raises(AssertionError):
        pins.test_fixed_point_trajectory_matches_library(_small())


def test_degenerate_counted_as_update_caught(monkeypatch):
    def fp(Xw, W0, tol, max_iter, traj_iters=0):
        B, iters, status, traj, ti = _fixed_point(Xw, W0, tol, max_iter, traj_iters)
        iters = iters + (status == ica.DEGENERATE)
        return B, iters, status, traj, ti
    monkeypatch.setattr(ica, "fixed_point", fp)
    with pytest.raises(AssertionError):
        pins.test_fixed_point_degenerate_rows(_small())
