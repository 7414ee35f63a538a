"""FP64 NumPy oracle of matrix-form ordering ICA -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import this module.  It never touches the HIP library.

Paper: Matsuda & Yamaguchi, "Efficient Estimation of Unique Components in
Independent Component Analysis by Matrix Representation" (arXiv 2408.17118).
Notation: the paper's N x M data matrix X is N x T here (T samples), its L
random starts are K rows here, and its iteration cap K is ``max_iter``.

Every array is float64.  Data are row-major: X is N x T (samples contiguous),
B and W are K x N (one candidate per row).  T is processed in blocks of
``TBLOCK`` samples so that the K x T matrix Z is never held whole; blocking only
splits the sums over samples, it changes no step of the method.

Where the paper is silent or garbled, the reading taken here is named in the
docstring (convergence test, shape of eq. 5, leftover rows, tie order, ...).
"""
from __future__ import annotations

import math

import numpy as np

TBLOCK = 1 << 14

# Per-row outcome codes (shared meaning with the C ABI, defined independently).
NOTCONV, CONV, PRUNED, DEGENERATE = 0, 1, 2, 3


class RankError(ValueError):
    """Covariance is singular (or numerically so): the data cannot be whitened."""


# ---------------------------------------------------------------------------
# Ordering criterion and Gaussianity test (Sec. 2.2, eqs. 1-3)
# ---------------------------------------------------------------------------

def upsilon(alpha):
    """Ordering criterion of eq. (1): alpha - 2 log(alpha/2 + 1).

    Defined for alpha > -2 (the log argument must be positive).  log1p keeps
    precision near alpha = 0, where the value behaves like alpha^2 / 4.  For
    alpha <= -2 the value is +inf (reading: the limit of the criterion as the
    log argument goes to 0+).  A unit-variance component has E y^4 >= (E y^2)^2,
    so alpha >= -2, with equality only for a +-1 (Bernoulli) variable, the one
    source Theorem 1 excludes.
    """
    a = np.asarray(alpha, dtype=np.float64)
    out = np.full(a.shape, np.inf)
    ok = a > -2.0
    out[ok] = a[ok] - 2.0 * np.log1p(a[ok] / 2.0)
    out[np.isnan(a)] = np.nan
    return out if out.ndim else float(out)


def gaussianity_threshold(N: int, i, T: int):
    """Right-hand side of the Gaussianity test, eq. (3): 2(N-i+2)(N-i+1)/T.

    ``i`` is the 1-based rank of the component being tested.  The components
    from rank i on are declared Gaussian once upsilon falls strictly below it.
    """
    i = np.asarray(i, dtype=np.float64)
    return 2.0 * (N - i + 2.0) * (N - i + 1.0) / float(T)


def kurtosis(Xw: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Kurtosis estimate of eq. (2) for every row b of B: sum_m (b.x_m)^4 / T - 3.

    Evaluated as written (no division by the sample variance): the rows of B
    are unit vectors and Xw is white, so y = bXw has unit sample variance.
    """
    B = np.atleast_2d(np.asarray(B, dtype=np.float64))
    N, T = Xw.shape
    s4 = np.zeros(B.shape[0])
    for m0 in range(0, T, TBLOCK):
        Z = B @ Xw[:, m0:m0 + TBLOCK]
        Z2 = Z * Z
        s4 += (Z2 * Z2).sum(axis=1)
    return s4 / T - 3.0


# ---------------------------------------------------------------------------
# Whitening (the data are whitened before the method runs, Sec. 2.2)
# ---------------------------------------------------------------------------

def whiten(X: np.ndarray, rank_tol: float = 1e-12):
    """PCA whitening so that the whitened rows satisfy the constraints of
    Theorem 1: zero sample mean and sample covariance I (normalised by T).

    Steps: mu = row means; Xc = X - mu; C = Xc Xc^T / T (divide by T, not T-1,
    because the theorem's constraint is sum_m y_i y_j / M = delta_ij);
    C = E D E^T with eigenvalues in descending order (stable for ties);
    each eigenvector's sign is fixed so that its entry of largest magnitude
    (lowest row on ties) is positive; V = D^(-1/2) E^T; Xw = V Xc.

    Raises RankError if the smallest eigenvalue is <= rank_tol * largest.
    Returns (Xw, V, mu, eigvals).
    """
    X = np.asarray(X, dtype=np.float64)
    N, T = X.shape
    mu = X.mean(axis=1)
    Xc = X - mu[:, None]
    C = (Xc @ Xc.T) / T
    lam, E = np.linalg.eigh(C)
    order = np.argsort(-lam, kind="stable")
    lam = lam[order]
    E = E[:, order]
    for j in range(N):
        p = int(np.argmax(np.abs(E[:, j])))
        if E[p, j] < 0:
            E[:, j] = -E[:, j]
    if not np.all(np.isfinite(lam)) or lam[-1] <= rank_tol * lam[0] or lam[0] <= 0:
        raise RankError(f"covariance is rank deficient (eigenvalues {lam[0]:.3e} .. {lam[-1]:.3e})")
    V = (E / np.sqrt(lam)).T
    Xw = V @ Xc
    return Xw, V, mu, lam


# ---------------------------------------------------------------------------
# The kurtosis fixed point
# ---------------------------------------------------------------------------

def normalise_rows(W: np.ndarray) -> np.ndarray:
    W = np.asarray(W, dtype=np.float64)
    return W / np.linalg.norm(W, axis=1, keepdims=True)


def update(Xw: np.ndarray, P: np.ndarray):
    """One matrix-form update before normalisation (Sec. 3.1, eqs. 4-5 as
    laid out in Algorithm 2): Z = P Xw, G = (Z o Z o Z) Xw^T / T - 3 P.

    Eq. (5) as printed multiplies in the transposed order (an N x L result for
    an L x N B); Algorithm 2's order, giving an L x N result, is the one taken.
    Also returns sum_m z^4 / T per row, i.e. eq. (2) + 3 for the rows of P.
    """
    N, T = Xw.shape
    G = np.zeros_like(P)
    s4 = np.zeros(P.shape[0])
    for m0 in range(0, T, TBLOCK):
        Xb = Xw[:, m0:m0 + TBLOCK]
        Z = P @ Xb
        Z3 = Z * Z * Z
        G += Z3 @ Xb.T
        s4 += (Z3 * Z).sum(axis=1)
    return G / T - 3.0 * P, s4 / T


def fixed_point(Xw: np.ndarray, W0: np.ndarray, tol: float, max_iter: int,
                traj_iters: int = 0):
    """Batched fixed point with removal of converged rows (Sec. 3.1-3.2 and
    the inner do-while of Algorithm 2).

    B starts as the row-normalised W0; every row is active.  Each pass takes
    the active rows P, forms G by ``update``, normalises each row, and measures
    the step d = min(||b - b_prev||, ||b + b_prev||).

    Readings:
      * Convergence: the paper's test combines the two distances with "or",
        which for unit vectors can never fail (their squares sum to 4).  A row
        is taken as converged when the smaller distance is strictly below tol;
        the "+" branch covers negative-kurtosis fixed points, where the iterate
        flips sign every pass.
      * The loop is a do-while: at least one update, at most max_iter passes.
      * A row whose G has zero or non-finite norm is DEGENERATE and keeps its
        previous value; rows still active after max_iter are NOTCONV.
      * iters[l] counts the updates applied to row l, including the one that
        converged it.
      * traj[l, t] = (alpha of the row before pass t+1, step d of pass t+1) for
        the first traj_iters passes; entries after a row stops are NaN.

    Returns (B, iters, status, traj, thread_iters) where thread_iters is the
    total number of row updates computed (sum over passes of active rows).
    """
    B = normalise_rows(W0).copy()
    K = B.shape[0]
    status = np.full(K, NOTCONV, dtype=np.uint8)
    iters = np.zeros(K, dtype=np.int64)
    traj = np.full((K, traj_iters, 2), np.nan)
    act = np.arange(K)
    t = 0
    thread_iters = 0
    while True:
        P = B[act]
        G, s4 = update(Xw, P)
        gn = np.linalg.norm(G, axis=1)
        ok = np.isfinite(gn) & (gn > 0.0)
        Bn = np.where(ok[:, None], G / np.where(ok, gn, 1.0)[:, None], P)
        d = np.minimum(np.linalg.norm(Bn - P, axis=1), np.linalg.norm(Bn + P, axis=1))
        if t < traj_iters:
            traj[act, t, 0] = s4 - 3.0
            traj[act, t, 1] = np.where(ok, d, np.nan)
        B[act] = Bn
        iters[act[ok]] += 1
        conv = ok & (d < tol)
        status[act[conv]] = CONV
        status[act[~ok]] = DEGENERATE
        thread_iters += len(act)
        act = act[ok & ~conv]
        t += 1
        if t >= max_iter or len(act) == 0:
            break
    return B, iters, status, traj, thread_iters


def fastica_single(Xw: np.ndarray, w0: np.ndarray, tol: float, max_iter: int):
    """Per-candidate form of the same fixed point: the FastICA function of
    Algorithm 1 with no projection (E = 0), run for one start vector.

    w is normalised; then repeatedly y = w^T Xw, w <- Xw y^3 / T - 3 w, w is
    normalised, until the step test of ``fixed_point`` passes or max_iter
    passes have run.  Returns (w, iters, converged).
    """
    N, T = Xw.shape
    w = np.asarray(w0, dtype=np.float64)
    w = w / math.sqrt(float(w @ w))
    t = 0
    while True:
        w_prev = w
        y = w @ Xw
        w = (Xw @ (y * y * y)) / T - 3.0 * w
        w = w / math.sqrt(float(w @ w))
        t += 1
        step = min(np.linalg.norm(w - w_prev), np.linalg.norm(w + w_prev))
        if step < tol:
            return w, t, True
        if t >= max_iter:
            return w, t, False


# ---------------------------------------------------------------------------
# Selection: clustering up to sign, ordering, Gaussianity test
# ---------------------------------------------------------------------------

def canonical_sign(v: np.ndarray) -> np.ndarray:
    """Flip v so that its entry of largest magnitude (lowest index on ties) is positive."""
    v = np.asarray(v, dtype=np.float64)
    p = int(np.argmax(np.abs(v)))
    return -v if v[p] < 0 else v.copy()


def unique(B: np.ndarray, alpha: np.ndarray, status: np.ndarray, T: int,
           tau: float = 1e-3, gaussianity_test: bool = True, n_top: int = 0):
    """Unique components from many converged candidates.

    Generalises Algorithm 2's argmax over candidates to the whole ordered set:
      1. Candidates are the CONV rows; if there are none, every non-degenerate
         row is used (the single-candidate FastICA of Algorithm 1 returns after
         max_iter passes whether or not it converged).
      2. Candidates are ordered by upsilon(alpha) descending, then row index.
      3. Greedy leader clustering up to sign: a candidate joins the first
         representative r with 1 - |b.b_r| <= tau, else it becomes a new
         representative.  The representative is the cluster's first member.
      4. Representatives keep that order (upsilon descending, then index) and
         are output with the canonical sign.
      5. Gaussianity walk (eq. 3 with the rank r in place of the deflation
         step): accept ranks 1, 2, ... while upsilon_r >= threshold(N, r, T);
         the first failure ends the walk.  Without the test every cluster is
         accepted.
      6. n_top > 0 truncates the accepted count.

    Returns a dict with U (n x N), alpha, upsilon, rep (row index), size,
    n_accepted.
    """
    B = np.asarray(B, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    status = np.asarray(status)
    K, N = B.shape
    ups = upsilon(alpha)
    cand = np.flatnonzero(status == CONV)
    if cand.size == 0:
        cand = np.flatnonzero(status != DEGENERATE)
    cand = cand[np.isfinite(alpha[cand])]
    order = cand[np.lexsort((cand, -ups[cand]))]
    reps: list[int] = []
    sizes: list[int] = []
    for l in order:
        for j, r in enumerate(reps):
            if 1.0 - abs(float(B[l] @ B[r])) <= tau:
                sizes[j] += 1
                break
        else:
            reps.append(int(l))
            sizes.append(1)
    reps_a = np.asarray(reps, dtype=np.int64)
    U = np.array([canonical_sign(B[r]) for r in reps]).reshape(len(reps), N)
    ups_u = ups[reps_a] if reps else np.zeros(0)
    n_acc = len(reps)
    if gaussianity_test:
        n_acc = 0
        for r in range(1, len(reps) + 1):
            if ups_u[r - 1] < gaussianity_threshold(N, r, T):
                break
            n_acc = r
    if n_top > 0:
        n_acc = min(n_acc, n_top)
    return {
        "U": U,
        "alpha": alpha[reps_a] if reps else np.zeros(0),
        "upsilon": ups_u,
        "rep": reps_a,
        "size": np.asarray(sizes, dtype=np.int64),
        "n_accepted": int(n_acc),
    }


def ordering_ica(X: np.ndarray, W0: np.ndarray, tol: float = 1e-10, max_iter: int = 1000,
                 tau: float = 1e-3, gaussianity_test: bool = True):
    """Whole hot path on raw data: whiten -> fixed point -> kurtosis -> unique.

    The unique components are also returned in raw-data space as unit rows
    u V (normalised), which survives rotations of the whitening basis inside
    near-degenerate eigenpairs.
    """
    Xw, V, mu, lam = whiten(X)
    B, iters, status, _, ti = fixed_point(Xw, W0, tol, max_iter)
    alpha = kurtosis(Xw, B)
    res = unique(B, alpha, status, Xw.shape[1], tau=tau, gaussianity_test=gaussianity_test)
    Ur = res["U"] @ V if len(res["U"]) else res["U"]
    if len(Ur):
        Ur = np.array([canonical_sign(u) for u in normalise_rows(Ur)])
    res.update(U_raw=Ur, B=B, iters=iters, status=status, kurt=alpha,
               thread_iters=ti, Xw=Xw, V=V, mu=mu, eigvals=lam)
    return res


def fluctuation(W_runs) -> np.ndarray:
    """Run-to-run fluctuation of Sec. 4.3: for component i, the mean over all
    ordered pairs (t, u), t != u, of 1 - |cos(w_i^t, w_i^u)|."""
    W_runs = [np.asarray(W, dtype=np.float64) for W in W_runs]
    R = len(W_runs)
    n = min(W.shape[0] for W in W_runs)
    out = np.zeros(n)
    for i in range(n):
        acc = 0.0
        for t in range(R):
            for u in range(R):
                if t == u:
                    continue
                a, b = W_runs[t][i], W_runs[u][i]
                acc += 1.0 - abs(float(a @ b)) / (np.linalg.norm(a) * np.linalg.norm(b))
        out[i] = acc / (R * (R - 1))
    return out


# ---------------------------------------------------------------------------
# The deflation driver: the outer loop of Algorithm 2 (Sec. 3.3, eqs. 6-8)
# ---------------------------------------------------------------------------

def reduce_basis(W: np.ndarray, N: int, rank_tol: float = 1e-12) -> np.ndarray:
    """Orthonormal basis of the complement of the rows of W (Sec. 3.3).

    F = I_N - W^T W (eq. 6); F~ keeps the first N - i + 1 rows of F, i.e.
    drops the bottom i - 1 rows, where i - 1 = W.shape[0] components are
    already estimated; G = (F~ F~^T)^(-1/2) F~ (eq. 7), the inverse square root
    taken from the eigendecomposition of the symmetric F~ F~^T.  With no
    component yet (i = 1), G = I_N.  Raises RankError when F~ F~^T is singular
    (smallest eigenvalue <= rank_tol x largest): the first N - i + 1 rows of F
    then do not span the complement.
    """
    W = np.asarray(W, dtype=np.float64).reshape(-1, N)
    n_prev = W.shape[0]
    if n_prev == 0:
        return np.eye(N)
    F = np.eye(N) - W.T @ W
    Ft = F[: N - n_prev]
    lam, E = np.linalg.eigh(Ft @ Ft.T)
    if not np.all(np.isfinite(lam)) or lam[0] <= rank_tol * lam[-1] or lam[-1] <= 0:
        raise RankError(f"F~ F~^T is singular (eigenvalues {lam[0]:.3e} .. {lam[-1]:.3e})")
    return (E / np.sqrt(lam)) @ E.T @ Ft


def deflation(Xw: np.ndarray, W0s, tol: float, max_iter: int, rank_tol: float = 1e-12,
              gaussianity_test: bool = True):
    """Fast ordering ICA, Algorithm 2: components one at a time.

    For step i = 1, 2, ...: G from the components found so far
    (``reduce_basis``), X~ = G Xw (eq. 8, an (N - i + 1) x T matrix); the batched
    fixed point with removal of converged rows from the start rows W0s[i-1]
    (L x (N - i + 1)); the kurtosis of every converged row on X~; p = the
    converged row of largest upsilon (lowest row index on ties; if no row
    converged, every non-degenerate row is a candidate, as in ``unique``).  If
    upsilon_p is below the Gaussianity threshold of eq. 3 for step i the loop
    ends (without the test, as in the EEG experiment of Sec. 4.3, all N steps
    run); otherwise the row b_p G (a unit vector in the whitened space,
    orthogonal to the earlier ones), re-orthogonalised against them to undo
    the rounding of eqs. 6-7, is appended to W.

    Returns (W, steps): W is n x N with the components in the order found;
    steps holds one dict per step taken (the last one may be the rejected step)
    with the dimension, p, alpha_p, upsilon_p, the threshold, whether it was
    accepted, and the fixed point's row updates.
    """
    N, T = Xw.shape
    W = np.zeros((0, N))
    steps = []
    for i in range(1, N + 1):
        G = reduce_basis(W, N, rank_tol)
        Xt = G @ Xw
        B, iters, status, _, ti = fixed_point(Xt, W0s[i - 1], tol, max_iter)
        cand = np.flatnonzero(status == CONV)
        if cand.size == 0:
            cand = np.flatnonzero(status != DEGENERATE)
        alpha = kurtosis(Xt, B[cand])
        ups = upsilon(alpha)
        k = int(np.argmax(ups))          # first maximum = lowest row index on ties
        p = int(cand[k])
        thr = float(gaussianity_threshold(N, i, T))
        ok = bool(ups[k] >= thr) or not gaussianity_test
        steps.append({"i": i, "dim": N - i + 1, "p": p, "alpha": float(alpha[k]),
                      "upsilon": float(ups[k]), "threshold": thr, "accepted": ok,
                      "thread_iters": int(ti), "n_conv": int(np.sum(status == CONV))})
        if not ok:
            break
        # b_p G is orthogonal to the rows of W in exact arithmetic; evaluated
        # as printed, the rounding of F~ and of the inverse square root
        # compounds from step to step (the rows of X~ must stay orthonormal to
        # the estimated components), so the row is orthogonalised against W
        # twice (classical Gram-Schmidt) before it is normalised
        w = B[p] @ G
        for _ in range(2):
            w = w - W.T @ (W @ w)
        W = np.vstack([W, w / np.linalg.norm(w)])
    return W, steps


def fastica_projected(Xw: np.ndarray, w0: np.ndarray, E: np.ndarray, tol: float, max_iter: int):
    """The FastICA function of Algorithm 1 with the projection E = W^T W of the
    components found so far: w <- w - E w and normalise, then repeatedly
    y = w^T Xw, w <- Xw y^3 / T - 3 w, w <- w - E w, normalise, until the step
    test of ``fixed_point`` passes or max_iter passes have run.
    Returns (w, iters, converged)."""
    w = np.asarray(w0, dtype=np.float64)
    w = w - E @ w
    w = w / math.sqrt(float(w @ w))
    T = Xw.shape[1]
    t = 0
    while True:
        w_prev = w
        y = w @ Xw
        w = (Xw @ (y * y * y)) / T - 3.0 * w
        w = w - E @ w
        w = w / math.sqrt(float(w @ w))
        t += 1
        step = min(np.linalg.norm(w - w_prev), np.linalg.norm(w + w_prev))
        if step < tol:
            return w, t, True
        if t >= max_iter:
            return w, t, False


def ordering_original(Xw: np.ndarray, W0s, tol: float, max_iter: int,
                      gaussianity_test: bool = True):
    """The original ordering ICA, Algorithm 1: for step i = 1, 2, ...,
    E = W^T W of the components found so far (0 at i = 1); every start row
    of W0s[i-1] (L x N) runs ``fastica_projected`` with E; the kurtosis of each
    returned vector; p = the run of largest upsilon over all runs (lowest index
    on ties; Algorithm 1 keeps every run, converged or not); the loop ends when
    upsilon_p is below eq. 3's threshold for step i (unless the test is off),
    else the vector of run p is appended to W.  Returns (W, steps) as
    ``deflation``."""
    N, T = Xw.shape
    W = np.zeros((0, N))
    steps = []
    for i in range(1, N + 1):
        E = W.T @ W if i > 1 else np.zeros((N, N))
        runs = [fastica_projected(Xw, w0, E, tol, max_iter) for w0 in W0s[i - 1]]
        V = np.array([r[0] for r in runs])
        alpha = kurtosis(Xw, V)
        ups = upsilon(alpha)
        p = int(np.argmax(ups))
        thr = float(gaussianity_threshold(N, i, T))
        ok = bool(ups[p] >= thr) or not gaussianity_test
        steps.append({"i": i, "dim": N, "p": p, "alpha": float(alpha[p]),
                      "upsilon": float(ups[p]), "threshold": thr, "accepted": ok,
                      "thread_iters": int(sum(r[1] for r in runs)),
                      "n_conv": int(sum(r[2] for r in runs))})
        if not ok:
            break
        W = np.vstack([W, V[p] / np.linalg.norm(V[p])])
    return W, steps
