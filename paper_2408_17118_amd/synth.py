"""Seeded synthetic workloads for matrix-form ordering ICA.

This module only draws numbers.  It holds none of the method's arithmetic: no
centring, whitening, kurtosis, fixed-point update or clustering.  Both the FP64
oracle (through the tests) and the GPU path (through the tests and the
benchmark) receive the arrays it returns, so the two sides always start from the
same data and the same random start vectors.

Data model (paper Sec. 2.1, the linear ICA model X = A S): S holds N independent
unit-variance sources of T samples each, A is an N x N mixing matrix with iid
N(0, 1) entries, and X = A S is the N x T observation matrix (row-major, samples
contiguous).  W0 is the K x N matrix of random start vectors (Algorithm 2 starts
from a random L x N matrix B); its entries are iid N(0, 1) rounded to FP32, so
that an FP32 device copy and an FP64 host copy hold exactly the same values.

Draw order for one problem, from one ``numpy.random.Generator``:
A (N x N, row-major), then the source rows in family order, then W0 (K x N).

Families (all unit variance, no per-sample standardisation):
  laplace   Laplace(0, 1/sqrt 2)
  student_t Student-t with nu degrees of freedom, scaled by sqrt((nu - 2)/nu)
  uniform   U(-sqrt 3, sqrt 3)
  sine      sqrt 2 * sin(2 pi f m + phi), f ~ U(1e-3, 5e-2) cycles/sample,
            phi ~ U(0, 2 pi), drawn per source before its samples
  gaussian  N(0, 1)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FAMILIES = ("laplace", "student_t", "uniform", "sine", "gaussian")

# Population excess kurtosis of each family (used by generator tests only).
def family_kurtosis(kind: str, nu: float = 5.0) -> float:
    if kind == "laplace":
        return 3.0
    if kind == "student_t":
        return 6.0 / (nu - 4.0) if nu > 4 else math.inf
    if kind == "uniform":
        return -1.2
    if kind == "sine":
        return -1.5
    if kind == "gaussian":
        return 0.0
    raise ValueError(kind)


def largest_remainder(total: int, ratios: list[float]) -> list[int]:
    """Split ``total`` into integer counts proportional to ``ratios``.

    Largest-remainder rounding; ties in the remainder go to the earlier entry.
    """
    s = float(sum(ratios))
    exact = [total * r / s for r in ratios]
    counts = [int(math.floor(e)) for e in exact]
    left = total - sum(counts)
    rem = [(-(e - c), i) for i, (e, c) in enumerate(zip(exact, counts))]
    rem.sort()
    for _, i in rem[:left]:
        counts[i] += 1
    return counts


# The mixed family ratio of the EEG-shaped workloads:
# laplace : student_t(nu=5) : uniform : sine : gaussian = 3 : 2 : 1.5 : 1 : 0.5
EEG_MIX = (3.0, 2.0, 1.5, 1.0, 0.5)


@dataclass
class Problem:
    """One seeded instance: observations, ground truth and start vectors."""

    X: np.ndarray          # N x T float64, X = A S
    A: np.ndarray          # N x N float64
    S: np.ndarray          # N x T float64
    W0: np.ndarray         # K x N float64 holding FP32-exact values (not normalised)
    kinds: list[str]       # family of each source row
    seed: object = None
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.X.shape[0]

    @property
    def T(self) -> int:
        return self.X.shape[1]

    @property
    def K(self) -> int:
        return self.W0.shape[0]


def draw_sources(rng: np.random.Generator, kinds: list[str], T: int, nu: float) -> np.ndarray:
    S = np.empty((len(kinds), T), dtype=np.float64)
    m = np.arange(T, dtype=np.float64)
    for i, kind in enumerate(kinds):
        if kind == "laplace":
            S[i] = rng.laplace(0.0, 1.0 / math.sqrt(2.0), T)
        elif kind == "student_t":
            S[i] = rng.standard_t(nu, T) * math.sqrt((nu - 2.0) / nu)
        elif kind == "uniform":
            S[i] = rng.uniform(-math.sqrt(3.0), math.sqrt(3.0), T)
        elif kind == "sine":
            f = rng.uniform(1e-3, 5e-2)
            phi = rng.uniform(0.0, 2.0 * math.pi)
            S[i] = math.sqrt(2.0) * np.sin(2.0 * math.pi * f * m + phi)
        elif kind == "gaussian":
            S[i] = rng.standard_normal(T)
        else:
            raise ValueError(f"unknown source family {kind!r}")
    return S


def draw_start(rng: np.random.Generator, K: int, N: int) -> np.ndarray:
    """K x N iid N(0,1) start vectors, rounded to FP32 and returned as float64."""
    return rng.standard_normal((K, N)).astype(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# Generalised Gaussian sources (the paper's artificial datasets, Sec. 4.2).
# ---------------------------------------------------------------------------

def gg_rhos(n_pos: int = 10, n_neg: int = 10) -> list[float]:
    """Shape parameters rho = 2 * 2^(i/4): i = -n_pos .. -1 (rho < 2, positive
    kurtosis) then i = 1 .. n_neg (rho > 2, negative kurtosis)."""
    return [2.0 * 2.0 ** (i / 4.0) for i in list(range(-n_pos, 0)) + list(range(1, n_neg + 1))]


def draw_gg(rng: np.random.Generator, rho: float, T: int) -> np.ndarray:
    """T samples of the generalised Gaussian with density proportional to
    exp(-(|u| / beta)^rho), beta chosen for unit variance: |u| / beta is
    G^(1/rho) with G ~ Gamma(1/rho, 1), with a random sign; the variance of
    G^(1/rho) is Gamma(3/rho) / Gamma(1/rho)."""
    g = rng.gamma(1.0 / rho, 1.0, T)
    sign = np.where(rng.random(T) < 0.5, -1.0, 1.0)
    scale = math.sqrt(math.gamma(1.0 / rho) / math.gamma(3.0 / rho))
    return sign * g ** (1.0 / rho) * scale


def artificial_gg(seed, n_gauss: int = 0, T: int = 10_000, K: int = 1) -> Problem:
    """The paper's artificial datasets: the 20 generalised Gaussian sources of
    ``gg_rhos`` (in that order) plus n_gauss N(0, 1) sources (0 for the first
    experiment, N = 20; 10 for the second, N = 30); A iid N(0, 1).  Draw order:
    A, the sources in order, W0 (K x N)."""
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    rhos = gg_rhos()
    N = len(rhos) + n_gauss
    A = rng.standard_normal((N, N))
    S = np.empty((N, T))
    for i, rho in enumerate(rhos):
        S[i] = draw_gg(rng, rho, T)
    for i in range(len(rhos), N):
        S[i] = rng.standard_normal(T)
    W0 = draw_start(rng, K, N)
    return Problem(X=A @ S, A=A, S=S, W0=W0,
                   kinds=[f"gg{r:.4f}" for r in rhos] + ["gaussian"] * n_gauss, seed=seed,
                   meta={"rhos": rhos, "T": T, "K": K})


def draw_deflation_starts(rng: np.random.Generator, L: int, N: int) -> list[np.ndarray]:
    """Start vectors of the deflation driver: for step i = 1..N an L x (N - i + 1)
    block of iid N(0,1) values rounded to FP32, drawn step after step from rng
    (Algorithm 2 draws a fresh random B at every step)."""
    return [draw_start(rng, L, N - i + 1) for i in range(1, N + 1)]


def draw_original_starts(rng: np.random.Generator, L: int, N: int) -> list[np.ndarray]:
    """Start vectors of Algorithm 1: an L x N block of iid N(0,1) values rounded
    to FP32 for each of the N steps, drawn step after step from rng."""
    return [draw_start(rng, L, N) for _ in range(N)]


def make_problem(kinds: list[str], T: int, K: int, seed, nu: float = 5.0) -> Problem:
    """Draw A, S and W0 for the given source families from one generator."""
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    N = len(kinds)
    A = rng.standard_normal((N, N))
    S = draw_sources(rng, kinds, T, nu)
    W0 = draw_start(rng, K, N)
    X = A @ S
    return Problem(X=X, A=A, S=S, W0=W0, kinds=list(kinds), seed=seed,
                   meta={"nu": nu, "T": T, "K": K})


def eeg_kinds(N: int, mix=EEG_MIX) -> list[str]:
    counts = largest_remainder(N, list(mix))
    kinds: list[str] = []
    for fam, c in zip(FAMILIES, counts):
        kinds += [fam] * c
    return kinds


# ---------------------------------------------------------------------------
# The five named workloads.
# ---------------------------------------------------------------------------

def small_mixture(seed: int = 0, K: int = 256, T: int = 10_000) -> Problem:
    """N=8, T=1e4: 4 Laplace, 2 uniform, 1 Student-t (nu=6), 1 Gaussian; K=256."""
    kinds = ["laplace"] * 4 + ["uniform"] * 2 + ["student_t"] + ["gaussian"]
    return make_problem(kinds, T=T, K=K, seed=seed, nu=6.0)


def eeg_shaped(seed: int = 1, N: int = 64, T: int = 200_000, K: int = 4096) -> Problem:
    """EEG-shaped mixture (N=64, T=2e5, K=4096): 24 Laplace, 16 t(nu=5),
    12 uniform, 8 sines, 4 Gaussian."""
    return make_problem(eeg_kinds(N), T=T, K=K, seed=seed, nu=5.0)


def precision_workload(seed: int = 3, N: int = 128, T: int = 1_000_000,
                       K: int = 16384) -> Problem:
    """N=128, T=1e6, K=16384 with the EEG-shaped family mix (48/32/24/16/8)."""
    return make_problem(eeg_kinds(N), T=T, K=K, seed=seed, nu=5.0)


def batched_shapes(seed: int = 4, D: int = 64, K: int = 1024,
                   t_lo: float = 2e4, t_hi: float = 5e5,
                   n_choices=tuple(range(16, 129, 8))):
    """Per-dataset (N_d, T_d, child generator) of the many-dataset workload.

    N_d is uniform over {16, 24, ..., 128}; T_d is log-uniform in [t_lo, t_hi].
    Each dataset draws from its own child of ``default_rng(seed).spawn(D)``.
    """
    children = np.random.default_rng(seed).spawn(D)
    out = []
    for rng in children:
        N = int(rng.choice(np.asarray(n_choices)))
        T = int(round(math.exp(rng.uniform(math.log(t_lo), math.log(t_hi)))))
        out.append((N, T, rng))
    return out


def batched_problem(N: int, T: int, rng: np.random.Generator, K: int = 1024) -> Problem:
    return make_problem(eeg_kinds(N), T=T, K=K, seed=rng, nu=5.0)


def pruner_workload(seed: int, N: int = 64, T: int = 200_000, K: int = 65536) -> Problem:
    """EEG-shaped mixture with K=65536 start vectors (training seeds 5000-5199,
    calibration 5200-5239, held-out test 5300-5319)."""
    return make_problem(eeg_kinds(N), T=T, K=K, seed=seed, nu=5.0)


WORKLOADS = {
    "small_mixture_n8": small_mixture,
    "eeg_shaped_n64": eeg_shaped,
    "precision_n128": precision_workload,
    "pruner_n64": pruner_workload,
}
