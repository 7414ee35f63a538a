"""Drivers of the paper's experiments (Sec. 4) on the GPU path.

Each driver runs the deflation driver (``Context.deflation``, Algorithm 2 of
the paper) through the C ABI and evaluates its output with the paper's
measures; the evaluation is plain host arithmetic on the returned components.

* ``artificial``: the generalised-Gaussian datasets of Sec. 4.2 -- 20 sources
  (N = 20, ordering error against the number of start rows L) or 20 sources
  plus 10 Gaussian ones (N = 30, the number of components the Gaussianity
  test accepts against L), T = 1e4, runs from different start rows, with the
  fast form (Algorithm 2) and the original one (Algorithm 1, batched).
* ``fluctuation``: the run-to-run fluctuation of Sec. 4.3 against L on one
  dataset (the Gaussianity test omitted, as there).

Run ``python -m paper_2408_17118_amd.studies`` for both on one GPU.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

from . import synth


def ordering_error(W_raw: np.ndarray, A: np.ndarray, source_order, thr: float = 0.1) -> float:
    """E_ordering = ||W A - I||_0 / N^2 (Sec. 4.2) with the sources sorted by
    their rank of non-Gaussianity (source_order[k] = the k-th source).  Rows of
    W A are normalised and an entry counts as nonzero when it differs from the
    identity's entry by more than thr in magnitude (a finite sample never gives
    exact zeros); missing rows (fewer components than N) count as zero rows."""
    N = A.shape[0]
    n = W_raw.shape[0]
    M = np.zeros((N, N))
    if n:
        C = np.abs(W_raw @ A[:, list(source_order)])
        M[:n] = C / np.linalg.norm(C, axis=1, keepdims=True)
    return float(np.count_nonzero(np.abs(M - np.eye(N)) > thr)) / float(N * N)


def fluctuation_delta(W_runs) -> np.ndarray:
    """Fluctuation of component i over runs (Sec. 4.3): the mean over ordered
    pairs of runs t != u of 1 - |cos(w_i^t, w_i^u)|, for the ranks every run
    reached."""
    R = len(W_runs)
    n = min(W.shape[0] for W in W_runs)
    U = np.stack([W[:n] / np.linalg.norm(W[:n], axis=1, keepdims=True) for W in W_runs])  # R x n x N
    cos = np.abs(np.einsum("tin,uin->tui", U, U))
    off = ~np.eye(R, dtype=bool)
    return (1.0 - cos[off]).mean(axis=0) if R > 1 else np.zeros(n)


def _upsilon(a):
    return a - 2.0 * np.log1p(a / 2.0)


def _source_order(S: np.ndarray):
    """Sources by descending criterion of their sample kurtosis (ties by index)."""
    Sc = S - S.mean(axis=1, keepdims=True)
    kap = (Sc ** 4).mean(axis=1) / (Sc ** 2).mean(axis=1) ** 2 - 3.0
    return sorted(range(S.shape[0]), key=lambda j: (-_upsilon(kap[j]), j))


def _deflate(ctx, Xw32, V, L, seed, gaussianity_test=True, precision="f32"):
    import torch
    N = Xw32.shape[0]
    starts = synth.draw_deflation_starts(np.random.default_rng(seed), L, N)
    flat = torch.from_numpy(np.concatenate([b.astype(np.float32).ravel() for b in starts])).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W, steps = ctx.deflation(Xw32, flat, precision=precision, gaussianity_test=gaussianity_test)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    Wr = (W @ V).cpu().numpy()
    if len(Wr):
        Wr /= np.linalg.norm(Wr, axis=1, keepdims=True)
    return Wr, steps, ms


def _original(ctx, Xw32, V, L, seed):
    import torch
    N = Xw32.shape[0]
    starts = synth.draw_original_starts(np.random.default_rng(seed), L, N)
    flat = torch.from_numpy(np.concatenate([b.astype(np.float32).ravel() for b in starts])).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W, steps = ctx.ordering_original(Xw32, flat)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    Wr = (W @ V).cpu().numpy()
    if len(Wr):
        Wr /= np.linalg.norm(Wr, axis=1, keepdims=True)
    return Wr, steps, ms


def artificial(ctx, n_gauss: int = 0, Ls=(1, 2, 5, 10, 20, 40, 60, 80, 100), runs: int = 10,
               data_seed: int = 0, start_seed: int = 1000, precision: str = "f32",
               original: bool = True):
    """Sec. 4.2 on one generated dataset: for every L, `runs` deflation runs
    from different start rows (and, with `original`, as many runs of
    Algorithm 1's batched variant for the fast-versus-original comparison).
    Returns one record per L with the mean and spread of the ordering error
    (n_gauss = 0) and of the number of accepted components, and the mean time
    per run of each form."""
    import torch
    prob = synth.artificial_gg(data_seed, n_gauss=n_gauss)
    X = torch.from_numpy(prob.X).cuda()
    Xw, Xw32, V, mean, eig = ctx.whiten(X)
    order = _source_order(prob.S)
    out = []
    for L in Ls:
        errs, found, times = [], [], []
        for r in range(runs):
            Wr, steps, ms = _deflate(ctx, Xw32, V, L, start_seed + 1000 * L + r, precision=precision)
            found.append(len(Wr))
            times.append(ms)
            if n_gauss == 0:
                errs.append(ordering_error(Wr, prob.A, order))
        rec = {"L": L, "runs": runs, "n_found_mean": float(np.mean(found)),
               "n_found": [int(f) for f in found], "ms_mean": float(np.mean(times))}
        if errs:
            rec.update(e_ordering_mean=float(np.mean(errs)), e_ordering_max=float(np.max(errs)))
        if original:
            o_err, o_found, o_ms = [], [], []
            for r in range(runs):
                Wr, steps, ms = _original(ctx, Xw32, V, L, start_seed + 1000 * L + r + 500)
                o_found.append(len(Wr))
                o_ms.append(ms)
                if n_gauss == 0:
                    o_err.append(ordering_error(Wr, prob.A, order))
            rec.update(original_ms_mean=float(np.mean(o_ms)),
                       original_n_found_mean=float(np.mean(o_found)))
            if o_err:
                rec.update(original_e_ordering_mean=float(np.mean(o_err)))
        out.append(rec)
    return {"N": prob.N, "T": prob.T, "n_gauss": n_gauss, "records": out}


def fluctuation(ctx, X, Ls=(10, 20, 40, 80, 120), runs: int = 10, start_seed: int = 5000,
                groups=((0, 20), (20, 40), (40, None))):
    """Sec. 4.3 on raw data X (device, N x T): for every L, `runs` deflation
    runs without the Gaussianity test; the fluctuation of each rank over the
    runs, averaged over all ranks and over the rank groups (1-20, 21-40, the
    rest)."""
    Xw, Xw32, V, mean, eig = ctx.whiten(X)
    out = []
    for L in Ls:
        Ws, times = [], []
        for r in range(runs):
            Wr, steps, ms = _deflate(ctx, Xw32, V, L, start_seed + 1000 * L + r, gaussianity_test=False)
            Ws.append(Wr)
            times.append(ms)
        d = fluctuation_delta(Ws)
        rec = {"L": L, "runs": runs, "delta_all": float(d.mean()), "ms_mean": float(np.mean(times)),
               "n_below_1e-6": int(np.sum(d <= 1e-6))}
        for a, b in groups:
            seg = d[a:b]
            rec[f"delta_{a + 1}-{b if b else len(d)}"] = float(seg.mean()) if len(seg) else None
        out.append(rec)
    return out


def main(argv=None):
    import torch

    from . import oica
    if not torch.cuda.is_available():
        print("the studies need a GPU", file=sys.stderr)
        return 1
    ctx = oica.Context(0)
    res = {"artificial_n20": artificial(ctx, 0), "artificial_n30": artificial(ctx, 10)}
    prob = synth.eeg_shaped()
    res["fluctuation_eeg_shaped_n64"] = fluctuation(ctx, torch.from_numpy(prob.X).cuda())
    print(json.dumps(res))
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
