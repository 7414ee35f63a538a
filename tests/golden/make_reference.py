"""Write the FP64 oracle's unique components for a named workload to a JSON
fixture.  Calls only the seeded generator and ``oracle/``.

Usage: python tests/golden/make_reference.py eeg_shaped_n64
       python tests/golden/make_reference.py precision_n128   (about 40 minutes)
       python tests/golden/make_reference.py batched_n16_128  (two datasets per
           padded-dimension class 32/64/96/128 of the 64-dataset workload)
       python tests/golden/make_reference.py batched_basins   (four datasets,
           one per padded-dimension class)
       python tests/golden/make_reference.py deflation_n24 | deflation_eeg_shaped_n64
           (the deflation driver, Algorithm 2's outer loop)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import ica  # noqa: E402
from paper_2408_17118_amd import synth  # noqa: E402

WORKLOADS = {
    "eeg_shaped_n64": lambda: synth.eeg_shaped(),
    "precision_n128": lambda: synth.precision_workload(),
}


def _entry(res, prob, dt, extra):
    out = {
        "N": prob.N, "T": prob.T, "K": prob.K, "tol": 1e-10, "max_iter": 1000, "tau": 1e-3,
        "oracle_seconds": dt, "thread_iters": int(res["thread_iters"]),
        "status_counts": [int((res["status"] == s).sum()) for s in range(4)],
        "n_unique": int(len(res["U"])), "n_accepted": int(res["n_accepted"]),
        "alpha": [float(a) for a in res["alpha"]],
        "upsilon": [float(u) for u in res["upsilon"]],
        "size": [int(s) for s in res["size"]],
        "rep": [int(r) for r in res["rep"]],
        "U_raw": [[float(v) for v in row] for row in res["U_raw"]],
    }
    out.update(extra)
    return out


# Datasets of the many-dataset workload checked against the oracle: the two
# with the smallest N T in each padded-dimension class (N rounded up to 32).
def batched_selection(shapes):
    by_class = {}
    for d, (N, T, _) in enumerate(shapes):
        by_class.setdefault((N + 31) // 32 * 32, []).append((N * T, d))
    return sorted(d for c in sorted(by_class) for _, d in sorted(by_class[c])[:2])


# One dataset per padded-dimension class with enough starts for every basin to
# be reached by at least six of them.
BASIN_SHAPES = [(20, 20_000, 1024, 300), (40, 20_000, 2048, 301), (80, 20_000, 4096, 302),
                (110, 20_000, 6144, 303)]


def main_many(name):
    entries = []
    if name == "batched_n16_128":
        shapes = synth.batched_shapes()
        todo = [(d, shapes[d]) for d in batched_selection(shapes)]
        probs = ((d, synth.batched_problem(N, T, rng)) for d, (N, T, rng) in todo)
    else:
        probs = ((d, synth.make_problem(synth.eeg_kinds(N), T=T, K=K, seed=seed))
                 for d, (N, T, K, seed) in enumerate(BASIN_SHAPES))
    for d, prob in probs:
        t0 = time.time()
        res = ica.ordering_ica(prob.X, prob.W0, tol=1e-10, max_iter=1000, tau=1e-3)
        dt = time.time() - t0
        entries.append(_entry(res, prob, dt, {"dataset": d}))
        print(f"dataset {d}: N={prob.N} T={prob.T} K={prob.K}: {len(res['U'])} clusters, "
              f"{res['n_accepted']} accepted, smallest {min(res['size'])}, {dt:.1f} s", flush=True)
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump({"workload": name, "datasets": entries}, f, indent=0)
    print(f"wrote {path}")


# Deflation driver runs: (data, start-row seed, L).  Both sides get the
# oracle's whitened data rounded to FP32 and the same start rows of every step.
DEFLATION = {
    "deflation_n24": (lambda: synth.make_problem(synth.eeg_kinds(24), T=50_000, K=8, seed=41), 42, 1024),
    "deflation_eeg_shaped_n64": (lambda: synth.eeg_shaped(), 43, 1024),
}


def main_deflation(name):
    import numpy as np
    make, seed, L = DEFLATION[name]
    prob = make()
    Xw, *_ = ica.whiten(prob.X)
    X32 = Xw.astype(np.float32).astype(np.float64)
    W0s = synth.draw_deflation_starts(np.random.default_rng(seed), L, prob.N)
    t0 = time.time()
    W, steps = ica.deflation(X32, W0s, 1e-10, 1000)
    dt = time.time() - t0
    out = {"workload": name, "N": prob.N, "T": prob.T, "L": L, "start_seed": seed,
           "tol": 1e-10, "max_iter": 1000, "oracle_seconds": dt, "n_found": int(W.shape[0]),
           "steps": steps, "W": [[float(v) for v in row] for row in W]}
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path}: {W.shape[0]} components in {len(steps)} steps, {dt:.1f} s")


def main(name):
    if name in ("batched_n16_128", "batched_basins"):
        return main_many(name)
    if name in DEFLATION:
        return main_deflation(name)
    prob = WORKLOADS[name]()
    t0 = time.time()
    res = ica.ordering_ica(prob.X, prob.W0, tol=1e-10, max_iter=1000, tau=1e-3)
    dt = time.time() - t0
    out = {
        "workload": name, "N": prob.N, "T": prob.T, "K": prob.K,
        "tol": 1e-10, "max_iter": 1000, "tau": 1e-3,
        "oracle_seconds": dt, "thread_iters": int(res["thread_iters"]),
        "status_counts": [int((res["status"] == s).sum()) for s in range(4)],
        "n_unique": int(len(res["U"])), "n_accepted": int(res["n_accepted"]),
        "alpha": [float(a) for a in res["alpha"]],
        "upsilon": [float(u) for u in res["upsilon"]],
        "size": [int(s) for s in res["size"]],
        "rep": [int(r) for r in res["rep"]],
        "U_raw": [[float(v) for v in row] for row in res["U_raw"]],
    }
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path}: {out['n_unique']} clusters, {out['n_accepted']} accepted, {dt:.1f} s")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "eeg_shaped_n64")
