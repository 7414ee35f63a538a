"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula and compares it with itself: each
check comes from an independent route -- closed forms evaluated elsewhere
(golden files), a library routine that implements the same update (scikit-learn
FastICA in deflation mode with the cube nonlinearity), scipy's kurtosis,
brute force over all directions at N = 2, algebraic identities of the update,
recovery of a known mixing matrix, and the paper's own run-to-run fluctuation.
"""
import math
import os

import numpy as np
import pytest

from oracle import ica
from paper_2408_17118_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


@pytest.fixture(scope="module")
def small():
    p = synth.small_mixture()
    Xw, V, mu, lam = ica.whiten(p.X)
    return p, Xw, V, mu, lam


# ---- P1: the ordering criterion (eq. 1) ------------------------------------

def test_upsilon_closed_forms():
    for a, v, *_ in _read_table("upsilon_closed_forms.txt"):
        assert ica.upsilon(float(a)) == pytest.approx(float(v), rel=1e-13, abs=1e-15)


def test_upsilon_series_near_zero():
    # Taylor series of a - 2 log(1 + a/2): a^2/4 - a^3/12 + a^4/32 - ...
    for a in (1e-3, -1e-3, 3e-2, -3e-2):
        series = a * a / 4 - a ** 3 / 12 + a ** 4 / 32 - a ** 5 / 80
        assert ica.upsilon(a) == pytest.approx(series, rel=1e-6)


def test_upsilon_shape():
    a = np.linspace(-1.99, 20, 4001)
    u = ica.upsilon(a)
    assert np.all(u >= 0)
    # derivative a / (2 + a): decreasing for a < 0, increasing for a > 0
    assert np.all(np.diff(u[a < 0]) < 0) and np.all(np.diff(u[a > 0]) > 0)
    assert ica.upsilon(-2.0) == math.inf and ica.upsilon(-3.0) == math.inf
    # sinusoids (-1.5) outrank Laplace (3): the criterion is not |kurtosis|
    assert ica.upsilon(-1.5) > ica.upsilon(3.0)


def test_gaussianity_threshold_table():
    for N, T, i, thr in _read_table("gaussianity_thresholds.txt"):
        assert ica.gaussianity_threshold(int(N), int(i), int(T)) == pytest.approx(float(thr), rel=1e-12)


# ---- P2: whitening ---------------------------------------------------------

def test_whiten_identity_covariance(small):
    p, Xw, V, mu, lam = small
    T = Xw.shape[1]
    assert np.max(np.abs(Xw @ Xw.T / T - np.eye(p.N))) < 1e-12
    assert np.max(np.abs(Xw.mean(axis=1))) < 1e-12
    Xc = p.X - p.X.mean(axis=1, keepdims=True)
    C = Xc @ Xc.T / T
    assert np.max(np.abs(V @ C @ V.T - np.eye(p.N))) < 1e-11
    assert np.all(np.diff(lam) <= 0)
    # canonical sign: largest-magnitude entry of every eigenvector (column of
    # V^T scaled) positive
    E = V.T * np.sqrt(lam)
    for j in range(p.N):
        assert E[np.argmax(np.abs(E[:, j])), j] > 0
    # eigenvalues agree with an SVD of the centred data (another LAPACK route)
    s = np.linalg.svd(Xc / math.sqrt(T), compute_uv=False)
    assert np.allclose(lam, s ** 2, rtol=1e-12)


def test_whiten_one_dimension():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((1, 5000)) * 3.0 + 2.0
    Xw, V, mu, lam = ica.whiten(x)
    assert np.allclose(Xw[0], (x[0] - x[0].mean()) / x[0].std(), atol=1e-13)


def test_whiten_rank_error():
    rng = np.random.default_rng(8)
    S = rng.standard_normal((3, 1000))
    X = np.vstack([S, S[:1]])          # duplicated row: singular covariance
    with pytest.raises(ica.RankError):
        ica.whiten(X)


# ---- P3, P7, P11: fixed-point invariants -----------------------------------

def test_fixed_point_unit_norm_and_status(small):
    p, Xw, *_ = small
    B, iters, status, traj, ti = ica.fixed_point(Xw, p.W0, tol=1e-10, max_iter=1000)
    assert np.max(np.abs(np.linalg.norm(B, axis=1) - 1.0)) < 1e-15 * 10
    assert np.all(status == ica.CONV)
    assert ti == int(iters.sum())


def test_update_identity(small):
    # <g + 3b, b> = sum_m (b.x_m)^4 / T exactly, for any unit b
    p, Xw, *_ = small
    P = ica.normalise_rows(p.W0[:32])
    G, s4 = ica.update(Xw, P)
    lhs = np.einsum("kn,kn->k", G + 3.0 * P, P)
    y = P @ Xw
    assert np.allclose(lhs, (y ** 4).mean(axis=1), rtol=1e-13)


def test_fixed_point_limits(small):
    # at a fixed point g = alpha b: ||g|| -> |alpha| and b . b_prev -> sign(alpha)
    p, Xw, *_ = small
    B, iters, status, *_ = ica.fixed_point(Xw, p.W0[:40], tol=1e-12, max_iter=1000)
    alpha = ica.kurtosis(Xw, B)
    G, _ = ica.update(Xw, B)
    gn = np.linalg.norm(G, axis=1)
    assert np.allclose(gn, np.abs(alpha), rtol=1e-9)
    cosines = np.einsum("kn,kn->k", G / gn[:, None], B)
    assert np.allclose(cosines, np.sign(alpha), atol=1e-9)


def test_matrix_form_equals_per_candidate_form(small):
    p, Xw, *_ = small
    W0 = p.W0[:24]
    B, iters, status, *_ = ica.fixed_point(Xw, W0, tol=1e-10, max_iter=1000)
    for l in range(W0.shape[0]):
        w, t, conv = ica.fastica_single(Xw, W0[l], tol=1e-10, max_iter=1000)
        assert conv == (status[l] == ica.CONV)
        assert t == iters[l]
        assert np.max(np.abs(w - B[l])) < 1e-12


# ---- P4: library FastICA (deflation, cube) ---------------------------------

def test_update_matches_library_fastica(small):
    sk = pytest.importorskip("sklearn.decomposition")
    p, Xw, *_ = small
    N = p.N
    W0 = p.W0[:N].copy()  # square start matrix; component 0 starts at W0[0]
    for n in (1, 2, 3, 6):
        ref = sk.FastICA(n_components=N, algorithm="deflation", whiten=False, fun="cube",
                         w_init=W0, max_iter=n, tol=0.0).fit(Xw.T).components_[0]
        w, t, conv = ica.fastica_single(Xw, W0[0], tol=0.0, max_iter=n)
        assert t == n
        assert np.max(np.abs(w - ref)) < 1e-12
        B, *_ = ica.fixed_point(Xw, W0[:1], tol=0.0, max_iter=n)
        assert np.max(np.abs(B[0] - ref)) < 1e-12


# ---- update's second output: sum z^4 / T (eq. 2 plus 3) ---------------------

def test_update_s4_matches_scipy(small):
    # scipy's non-excess kurtosis m4 / m2^2 uses central moments; for unit rows
    # on white, centred data m2 = 1 and the mean is 0, so it equals sum z^4 / T
    scipy_stats = pytest.importorskip("scipy.stats")
    p, Xw, *_ = small
    P = ica.normalise_rows(p.W0[:32])
    _, s4 = ica.update(Xw, P)
    ref = scipy_stats.kurtosis(P @ Xw, axis=1, fisher=False, bias=True)
    assert np.allclose(s4, ref, rtol=1e-10, atol=0.0)


# ---- the recorded trajectory against library FastICA iterates ---------------

def _library_iterates(Xw, w_first, others, n):
    """Iterates w_0 .. w_n of component 0 of scikit-learn's FastICA (deflation,
    cube, no whitening, tol 0) started from w_first: w_t is the fit with
    max_iter = t (w_0 is the normalised start)."""
    import warnings

    sk = pytest.importorskip("sklearn.decomposition")
    w_init = np.vstack([w_first, others])
    out = [w_first / np.linalg.norm(w_first)]
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        for t in range(1, n + 1):
            out.append(sk.FastICA(n_components=w_init.shape[0], algorithm="deflation",
                                  whiten=False, fun="cube", w_init=w_init, max_iter=t,
                                  tol=0.0).fit(Xw.T).components_[0])
    return out


def test_fixed_point_trajectory_matches_library(small):
    # traj[l, t] = (excess kurtosis of the row before pass t+1, step of pass t+1):
    # the kurtosis from scipy on the library's iterate w_t, the step
    # min(||w_{t+1} - w_t||, ||w_{t+1} + w_t||) from the library's iterates
    scipy_stats = pytest.importorskip("scipy.stats")
    p, Xw, *_ = small
    N = p.N
    rows = [0, 5, 17, 100, 201]
    R = 20
    B, iters, status, traj, _ = ica.fixed_point(Xw, p.W0[rows], tol=1e-10, max_iter=1000,
                                                traj_iters=R)
    stopped_early = 0
    for i, l in enumerate(rows):
        others = np.delete(p.W0[:N], 0, axis=0)
        ws = _library_iterates(Xw, p.W0[l], others[: N - 1], min(R, int(iters[i])))
        for t in range(R):
            if t >= iters[i]:
                # passes after the row stopped are not recorded
                assert np.isnan(traj[i, t, 0]) and np.isnan(traj[i, t, 1])
                stopped_early += 1
                continue
            a_ref = scipy_stats.kurtosis(ws[t] @ Xw, fisher=True, bias=True)
            d_ref = min(np.linalg.norm(ws[t + 1] - ws[t]), np.linalg.norm(ws[t + 1] + ws[t]))
            assert abs(traj[i, t, 0] - a_ref) < 1e-10, (l, t)
            assert abs(traj[i, t, 1] - d_ref) < 1e-11, (l, t)
    assert stopped_early > 0      # the NaN tail is exercised


# ---- R17: degenerate rows -----------------------------------------------------

def test_fixed_point_degenerate_rows(small):
    # a zero or non-finite start row has no direction: it is DEGENERATE with
    # no update applied; every other row evolves exactly as it would alone
    p, Xw, *_ = small
    W0 = p.W0[:16].copy()
    W0[3] = 0.0
    W0[9, 2] = np.nan
    with np.errstate(invalid="ignore", divide="ignore"):
        B, iters, status, traj, ti = ica.fixed_point(Xw, W0, tol=1e-10, max_iter=1000,
                                                     traj_iters=4)
    for l in (3, 9):
        assert status[l] == ica.DEGENERATE and iters[l] == 0
        assert np.all(np.isnan(traj[l, :, 1]))
    good = [l for l in range(16) if l not in (3, 9)]
    B2, iters2, status2, *_ = ica.fixed_point(Xw, W0[good], tol=1e-10, max_iter=1000)
    assert np.array_equal(iters[good], iters2) and np.array_equal(status[good], status2)
    assert np.max(np.abs(B[good] - B2)) < 1e-12
    assert np.all(status2 == ica.CONV)
    # the single-candidate form agrees on the surviving rows
    for i, l in enumerate(good[:4]):
        w, t, conv = ica.fastica_single(Xw, W0[l], tol=1e-10, max_iter=1000)
        assert conv and t == iters2[i] and np.max(np.abs(w - B2[i])) < 1e-12


# ---- P5: brute force over all directions at N = 2 ---------------------------

def _alpha_on_circle(Xw, theta):
    # E[(c x1 + s x2)^4] expanded by the binomial theorem in the five fourth
    # moments of the data; a route independent of the oracle's kurtosis().
    x1, x2 = Xw
    M = [np.mean(x1 ** (4 - k) * x2 ** k) for k in range(5)]
    c, s = np.cos(theta), np.sin(theta)
    e4 = c ** 4 * M[0] + 4 * c ** 3 * s * M[1] + 6 * c ** 2 * s ** 2 * M[2] \
        + 4 * c * s ** 3 * M[3] + s ** 4 * M[4]
    return e4 - 3.0


def _golden_max(f, a, b, tol=1e-10):
    g = (math.sqrt(5) - 1) / 2
    c, d = b - g * (b - a), a + g * (b - a)
    while b - a > tol:
        if f(c) > f(d):
            b, d = d, c
            c = b - g * (b - a)
        else:
            a, c = c, d
            d = a + g * (b - a)
    return 0.5 * (a + b)


@pytest.mark.parametrize("pair", [("laplace", "uniform"), ("student_t", "sine"), ("uniform", "sine")])
def test_two_dimensional_sweep(pair):
    prob = synth.make_problem(list(pair), T=20000, K=64, seed=11, nu=6.0)
    Xw, *_ = ica.whiten(prob.X)
    th = np.linspace(0.0, math.pi, 200_000, endpoint=False)
    ups = ica.upsilon(_alpha_on_circle(Xw, th))
    n = len(th)
    is_max = (ups > np.roll(ups, 1)) & (ups >= np.roll(ups, -1))
    maxima = []
    for i in np.flatnonzero(is_max):
        f = lambda t: float(ica.upsilon(_alpha_on_circle(Xw, np.array([t]))[0]))
        t0 = _golden_max(f, th[i] - 2 * math.pi / n, th[i] + 2 * math.pi / n)
        maxima.append(t0 % math.pi)
    assert 1 <= len(maxima) <= 4
    B, iters, status, *_ = ica.fixed_point(Xw, prob.W0, tol=1e-10, max_iter=1000)
    alpha = ica.kurtosis(Xw, B)
    for l in range(B.shape[0]):
        assert status[l] == ica.CONV
        ang = math.atan2(B[l, 1], B[l, 0]) % math.pi
        dist = [min(abs(ang - m), math.pi - abs(ang - m)) for m in maxima]
        j = int(np.argmin(dist))
        assert dist[j] < 1e-6
        assert alpha[l] == pytest.approx(float(_alpha_on_circle(Xw, np.array([maxima[j]]))[0]), abs=1e-9)


# ---- P6: N = 1 --------------------------------------------------------------

def test_one_dimension_fixed_point():
    scipy_stats = pytest.importorskip("scipy.stats")
    rng = np.random.default_rng(3)
    x = rng.laplace(size=(1, 4000))
    Xw, *_ = ica.whiten(x)
    W0 = np.array([[0.3], [-2.0], [1.0]])
    B, iters, status, *_ = ica.fixed_point(Xw, W0, tol=1e-10, max_iter=50)
    assert np.all(status == ica.CONV) and np.all(iters == 1)
    assert np.allclose(np.abs(B), 1.0)
    alpha = ica.kurtosis(Xw, B)
    assert np.allclose(alpha, scipy_stats.kurtosis(x[0], fisher=True, bias=True), rtol=1e-12)


# ---- P8: kurtosis against scipy ---------------------------------------------

def test_kurtosis_matches_scipy(small):
    scipy_stats = pytest.importorskip("scipy.stats")
    p, Xw, *_ = small
    B = ica.normalise_rows(p.W0[:16])
    ref = scipy_stats.kurtosis(B @ Xw, axis=1, fisher=True, bias=True)
    assert np.allclose(ica.kurtosis(Xw, B), ref, rtol=1e-11, atol=1e-12)


# ---- P9: recovery of the known mixing matrix, in Upsilon order -------------

def test_recovery_small_mixture(small):
    p = small[0]
    res = ica.ordering_ica(p.X, p.W0, tol=1e-10, max_iter=1000)
    n_ng = sum(k != "gaussian" for k in p.kinds)
    assert res["n_accepted"] == n_ng
    C = res["U_raw"][: res["n_accepted"]] @ p.A    # rows ~ +-e_j: a signed permutation
    purity = np.max(np.abs(C), axis=1) / np.linalg.norm(C, axis=1)
    assert np.all(purity >= 0.99)
    matched = np.argmax(np.abs(C), axis=1)
    assert sorted(matched) == [j for j, k in enumerate(p.kinds) if k != "gaussian"]
    # order: descending Upsilon of the true sources' sample kurtosis
    S = p.S - p.S.mean(axis=1, keepdims=True)
    kap = (S ** 4).mean(axis=1) / (S ** 2).mean(axis=1) ** 2 - 3
    expect = sorted(matched, key=lambda j: -ica.upsilon(kap[j]))
    assert list(matched) == expect
    assert np.all(np.diff(res["upsilon"]) <= 0)


def test_unique_components_are_orthonormal(small):
    p = small[0]
    res = ica.ordering_ica(p.X, p.W0, tol=1e-10, max_iter=1000)
    U = res["U"]
    # distinct fixed points are orthogonal up to O(T^-1/2) sampling error
    assert np.max(np.abs(U @ U.T - np.eye(len(U)))) < 0.1


# ---- P10: run-to-run fluctuation (Sec. 4.3) ---------------------------------

@pytest.mark.slow
def test_fluctuation_across_start_seeds(small):
    p, Xw, *_ = small
    runs = []
    for s in range(10):
        W0 = synth.draw_start(np.random.default_rng(100 + s), 256, p.N)
        B, it, st, *_ = ica.fixed_point(Xw, W0, tol=1e-10, max_iter=1000)
        res = ica.unique(B, ica.kurtosis(Xw, B), st, Xw.shape[1])
        runs.append(res["U"][: res["n_accepted"]])
    assert len({len(r) for r in runs}) == 1
    delta = ica.fluctuation(runs)
    assert np.all(delta <= 1e-6)


def test_fluctuation_extremes():
    a = np.array([[1.0, 0.0]])
    assert ica.fluctuation([a, -a]) == pytest.approx([0.0])
    assert ica.fluctuation([a, np.array([[0.0, 1.0]])]) == pytest.approx([1.0])


# ---- clustering and the Gaussianity walk on planted inputs -------------------

def _planted(seed=5, N=12, n_clusters=6, per=7, noise=1e-6):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    rows, labels = [], []
    for c in range(n_clusters):
        for _ in range(per):
            v = Q[c] + noise * rng.standard_normal(N)
            v = v / np.linalg.norm(v) * rng.choice([-1.0, 1.0])
            rows.append(v)
            labels.append(c)
    perm = rng.permutation(len(rows))
    return np.array(rows)[perm], np.array(labels)[perm], Q


def test_unique_planted_clusters():
    B, labels, Q = _planted()
    K = len(labels)
    # cluster c gets kurtosis 6 - c (distinct per cluster, tiny spread inside)
    rng = np.random.default_rng(1)
    alpha = 6.0 - labels + 1e-9 * rng.standard_normal(K)
    status = np.full(K, ica.CONV, dtype=np.uint8)
    res = ica.unique(B, alpha, status, T=10_000, tau=1e-3, gaussianity_test=False)
    assert len(res["U"]) == 6 and res["n_accepted"] == 6
    assert list(res["size"]) == [7] * 6
    for c in range(6):   # clusters come out in descending kurtosis = label order
        assert abs(res["U"][c] @ Q[c]) > 1 - 1e-9
        members = np.flatnonzero(labels == c)
        best = members[np.lexsort((members, -ica.upsilon(alpha[members])))[0]]
        assert res["rep"][c] == best
        u = res["U"][c]
        assert u[np.argmax(np.abs(u))] > 0


def test_unique_brute_force_partition():
    # any tau in the gap between within-cluster (~1e-12) and across-cluster (~1)
    # distances gives the connected components of the |cos| graph
    B, labels, Q = _planted(seed=9, noise=1e-5)
    K = len(labels)
    status = np.full(K, ica.CONV, dtype=np.uint8)
    alpha = np.linspace(5, 1, K)
    for tau in (1e-8, 1e-3, 1e-1):
        res = ica.unique(B, alpha, status, T=1000, tau=tau, gaussianity_test=False)
        assert sorted(res["size"]) == [7] * 6


def test_unique_excludes_unconverged_and_degenerate():
    B, labels, Q = _planted(seed=2, n_clusters=3, per=4)
    K = len(labels)
    status = np.full(K, ica.CONV, dtype=np.uint8)
    status[labels == 2] = ica.NOTCONV
    alpha = np.full(K, 3.0)
    res = ica.unique(B, alpha, status, T=1000, gaussianity_test=False)
    assert len(res["U"]) == 2
    status[:] = ica.NOTCONV           # none converged: every row is used
    status[0] = ica.DEGENERATE
    res = ica.unique(B, alpha, status, T=1000, gaussianity_test=False)
    assert len(res["U"]) == 3 and res["size"].sum() == K - 1


def test_gaussianity_walk():
    # N = 4, T = 100: thresholds 0.4, 0.24, 0.12, 0.04 (eq. 3, golden table)
    N, T = 4, 100
    Q = np.eye(N)

    def inv(u):   # alpha > 0 with upsilon(alpha) = u, by bisection
        lo, hi = 0.0, 50.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if ica.upsilon(mid) < u else (lo, mid)
        return hi

    status = np.full(N, ica.CONV, dtype=np.uint8)
    # ranks 1..4 get 0.9, 0.5, 0.3, 0.11: all above 0.4, 0.24, 0.12, 0.04
    alpha = np.array([inv(u) for u in (0.5, 0.3, 0.11, 0.9)])
    res = ica.unique(Q, alpha, status, T=T)
    assert np.allclose(res["upsilon"], [0.9, 0.5, 0.3, 0.11], rtol=1e-9)
    assert res["n_accepted"] == 4
    # ranks 1..4 get 0.5, 0.3, 0.11, 0.05: rank 3 fails (0.11 < 0.12) and ends
    # the walk even though rank 4 would pass its own threshold
    alpha = np.array([inv(u) for u in (0.5, 0.3, 0.11, 0.05)])
    res = ica.unique(Q, alpha, status, T=T)
    assert res["n_accepted"] == 2
    # the walk breaks on "<": a value at (or just above) the threshold passes
    res = ica.unique(Q[:1], np.array([inv(0.4)]), status[:1], T=T)
    assert res["n_accepted"] == 1
    res = ica.unique(Q[:1], np.array([inv(0.4) * (1 - 1e-9)]), status[:1], T=T)
    assert res["n_accepted"] == 0
    res = ica.unique(Q, np.array([inv(u) for u in (0.5, 0.3, 0.2, 0.9)]), status, T=T, n_top=1)
    assert res["n_accepted"] == 1
