"""The allocation-free entry point oica_kurtosis_noalloc against oica_kurtosis.

Both run the same kernels, so the results must be bitwise equal; both are also
held to the oracle's kurtosis (eq. 2) at the parity tolerance.  Two calls in a
row, the second smaller, show that the shared fixed array carries nothing over
from one call to the next.  A size beyond the array is refused on the host.
"""
import numpy as np
import pytest

from oracle import ica
from paper_2408_17118_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_noalloc_matches_the_allocating_call():
    from paper_2408_17118_amd import oica
    ctx = oica.Context(0)
    for N, T, K, seed in ((64, 50_000, 3000, 21), (17, 9_999, 70, 22)):
        print(f"noalloc kurtosis N={N} T={T} K={K} seed={seed}", flush=True)
        p = synth.make_problem(synth.eeg_kinds(N), T=T, K=K, seed=seed)
        Xw, *_ = ica.whiten(p.X)
        X32 = Xw.astype(np.float32)
        W = ica.normalise_rows(p.W0).astype(np.float32)
        Xd, Wd = torch.from_numpy(X32).cuda(), torch.from_numpy(W).cuda()
        ref = ctx.kurtosis(Xd, Wd)
        k = torch.full((K,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.kurtosis_noalloc(Xd, Wd, k)
        torch.cuda.synchronize()
        assert torch.equal(k, ref)
        kr = ica.kurtosis(X32.astype(np.float64), W.astype(np.float64))
        kg = k.cpu().numpy()
        assert np.all(np.abs(kg - kr) <= 1e-5 * np.maximum(np.abs(kr), 0.1))
    # more rows than the fixed array has partial sums for: refused before any launch
    Kbig = 2_200_000
    X1 = torch.ones((1, 4), dtype=torch.float32, device="cuda")
    Wbig = torch.ones((Kbig, 1), dtype=torch.float32, device="cuda")
    kbig = torch.empty(Kbig, dtype=torch.float64, device="cuda")
    with pytest.raises(oica.OicaError) as e:
        ctx.kurtosis_noalloc(X1, Wbig, kbig)
    assert e.value.code == -7          # OICA_E_UNSUPPORTED
    ctx.close()
