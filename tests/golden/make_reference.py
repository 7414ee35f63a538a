"""Write the FP64 oracle's unique components for a named workload to a JSON
fixture.  Calls only the seeded generator and ``oracle/``.

Usage: python tests/golden/make_reference.py eeg_shaped_n64
       python tests/golden/make_reference.py precision_n128   (about an hour)
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


def main(name):
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
