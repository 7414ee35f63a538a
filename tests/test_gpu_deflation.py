"""The deflation driver (Algorithm 2's outer loop, Sec. 3.3, eqs. 6-8) through
oica_deflation, against the oracle's driver on the same whitened data (the
oracle's, rounded to FP32) and the same start rows of every step.

Per step: the same dimension, the accepted flag and eq. 3's threshold; the
component at |cos| >= 1 - 1e-6 with the oracle's (whitened space) and its
kurtosis within 1e-5 max(|alpha|, 0.1).  The small mixture runs the oracle
live; the EEG-shaped family mix at N = 24 and the EEG-shaped workload
(N = 64, T = 2e5, 1024 starts per step) compare with stored oracle runs
(tests/golden/deflation_*_oracle.json, written by make_reference.py).  The chosen start row itself may
differ inside one cluster (its members' criterion values agree to FP32
rounding).  The GPU's components are orthonormal.
"""
import numpy as np
import pytest

from oracle import ica
from paper_2408_17118_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2408_17118_amd import oica
    c = oica.Context(0)
    yield c
    c.close()


def _compare(ctx, p, L, seed, precision="f32"):
    Xw, *_ = ica.whiten(p.X)
    X32 = Xw.astype(np.float32)
    W0s = synth.draw_deflation_starts(np.random.default_rng(seed), L, p.N)
    Wr, steps_r = ica.deflation(X32.astype(np.float64), W0s, 1e-10, 1000)
    Wg, steps_g = ctx.deflation(torch.from_numpy(X32).cuda(),
                                [torch.from_numpy(b.astype(np.float32)).cuda() for b in W0s],
                                tol=1e-6, max_iter=1000, precision=precision)
    Wg = Wg.cpu().numpy()
    print(f"N={p.N} T={p.T} L={L} {precision}: gpu {len(Wg)} components / {len(steps_g)} steps, "
          f"oracle {len(Wr)} / {len(steps_r)}")
    assert len(steps_g) == len(steps_r)
    assert len(Wg) == len(Wr)
    for sg, sr in zip(steps_g, steps_r):
        assert sg["dim"] == sr["dim"]
        assert sg["threshold"] == pytest.approx(sr["threshold"], rel=1e-12)
        assert bool(sg["accepted"]) == sr["accepted"], (sg, sr)
        assert abs(sg["alpha"] - sr["alpha"]) <= 1e-5 * max(abs(sr["alpha"]), 0.1), (sg, sr)
    cos = np.abs(np.einsum("kn,kn->k", Wg, Wr))
    print(f"  1-|cos| max {np.max(1 - cos) if len(cos) else 0:.3e}")
    assert np.all(cos >= 1 - 1e-6), np.flatnonzero(cos < 1 - 1e-6)
    assert np.max(np.abs(Wg @ Wg.T - np.eye(len(Wg)))) < 1e-12
    return Wg, steps_g


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_small_mixture(ctx, precision):
    p = synth.small_mixture()
    _compare(ctx, p, 256, 10, precision)


def _compare_golden(ctx, name):
    import json
    import os
    import sys
    gold = os.path.join(os.path.dirname(__file__), "golden")
    sys.path.insert(0, gold)
    import make_reference as mr
    ref = json.load(open(os.path.join(gold, f"{name}_oracle.json")))
    make, seed, L = mr.DEFLATION[name]
    p = make()
    Xw, *_ = ica.whiten(p.X)
    X32 = Xw.astype(np.float32)
    W0s = synth.draw_deflation_starts(np.random.default_rng(seed), L, p.N)
    Wg, steps_g = ctx.deflation(torch.from_numpy(X32).cuda(),
                                [torch.from_numpy(b.astype(np.float32)).cuda() for b in W0s],
                                tol=1e-6, max_iter=1000)
    Wg = Wg.cpu().numpy()
    Wr = np.asarray(ref["W"])
    steps_r = ref["steps"]
    print(f"{name}: gpu {len(Wg)} components / {len(steps_g)} steps, oracle {len(Wr)} / {len(steps_r)}")
    assert len(steps_g) == len(steps_r) and len(Wg) == len(Wr)
    for sg, sr in zip(steps_g, steps_r):
        assert sg["dim"] == sr["dim"]
        assert bool(sg["accepted"]) == sr["accepted"], (sg, sr)
        assert abs(sg["alpha"] - sr["alpha"]) <= 1e-5 * max(abs(sr["alpha"]), 0.1), (sg, sr)
    cos = np.abs(np.einsum("kn,kn->k", Wg, Wr))
    print(f"  1-|cos| max {np.max(1 - cos):.3e}")
    assert np.all(cos >= 1 - 1e-6), np.flatnonzero(cos < 1 - 1e-6)
    # (F~ F~^T)^(-1/2) amplifies rounding along the found components when the
    # kept rows of F are nearly dependent, so late components lose some
    # orthogonality in FP64 too: held to the oracle's own deviation
    dev_g = np.max(np.abs(Wg @ Wg.T - np.eye(len(Wg))))
    dev_r = np.max(np.abs(Wr @ Wr.T - np.eye(len(Wr))))
    print(f"  orthonormality: gpu {dev_g:.2e}, oracle {dev_r:.2e}")
    assert dev_g <= 10 * dev_r + 1e-12


def test_eeg_family_mix_n24(ctx):
    # the EEG-shaped family mix at N = 24 (9 Laplace, 6 t, 5 uniform, 3 sines, 1 Gaussian)
    _compare_golden(ctx, "deflation_n24")


@pytest.mark.slow
def test_eeg_shaped_n64(ctx):
    _compare_golden(ctx, "deflation_eeg_shaped_n64")
