"""The experiment drivers' measures (Sec. 4), on the CPU: the fluctuation of
Sec. 4.3 against the oracle's, and the ordering error of Sec. 4.2 on planted
separating matrices."""
import numpy as np

from oracle import ica
from paper_2408_17118_amd import studies


def test_fluctuation_matches_oracle():
    rng = np.random.default_rng(3)
    base = rng.standard_normal((6, 9))
    runs = [base * rng.choice([-1.0, 1.0], size=(6, 1)) + 1e-3 * rng.standard_normal((6, 9))
            for _ in range(4)]
    runs[2] = runs[2][:5]                    # one run reached fewer ranks
    d = studies.fluctuation_delta(runs)
    assert len(d) == 5
    assert np.allclose(d, ica.fluctuation(runs), rtol=1e-12, atol=1e-15)


def test_ordering_error_planted():
    rng = np.random.default_rng(4)
    N = 7
    A = rng.standard_normal((N, N))
    order = list(rng.permutation(N))
    W = np.linalg.inv(A)[order] * rng.choice([-2.0, 0.5], size=(N, 1))   # exact, in rank order
    assert studies.ordering_error(W, A, order) == 0.0
    Ws = W.copy()
    Ws[[1, 4]] = Ws[[4, 1]]                  # two components swapped: 4 wrong entries
    assert studies.ordering_error(Ws, A, order) == 4 / N ** 2
    assert studies.ordering_error(W[:-1], A, order) == 1 / N ** 2   # the last one missing
    C = W @ A                                 # a signed, scaled permutation
    Cn = C + 0.01 * np.abs(C).max(axis=1, keepdims=True) * rng.standard_normal(C.shape)
    assert studies.ordering_error(Cn @ np.linalg.inv(A), A, order) == 0.0
