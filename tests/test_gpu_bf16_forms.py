"""The three row forms of the BF16 passes (bf16_row_terms): 1 = the row rounded
once to BF16 and the linear term on the same rounded row, 2 = hi + lo BF16
parts with the linear term on the FP32 row, 3 = form 1 while a row's last
step is large, then form 2, 4 = form 2 while the step is large, then form 1;
0 = the default (form 2; the Python entry points default to tol_bf16 = 1e-3).

* One pass of form 1 is the update (eqs. 4-5) of the BF16-rounded row: its
  output equals the normalised G of the single-update entry point given the
  rounded rows (where the lo part is zero, so the products are the same),
  and it is within the z^3-rounding bound of the oracle's update of the
  rounded row on the same BF16 data.  The same output with the linear term
  taken on the unrounded row differs by far more than the tolerance, so the
  check sees which row the linear term used.
* Every form, followed by the FP32 finish, gives the oracle's unique set on
  the EEG-shaped workload (N=64, T=2e5, K=16384; golden from
  tests/golden/make_reference.py).
"""
import json
import os

import numpy as np
import pytest

from oracle import ica
from paper_2408_17118_amd import synth
from tests.test_gpu_bf16 import _check_against, bf16_round, dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2408_17118_amd import oica
    c = oica.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("N,T,K", [(8, 10_000, 256), (64, 20_000, 300), (128, 12_347, 129),
                                   (40, 5_003, 77)])
def test_one_term_pass_is_update_of_rounded_row(ctx, N, T, K):
    p = synth.make_problem(synth.eeg_kinds(N), T=T, K=K, seed=N * 7 + 2)
    Xw, *_ = ica.whiten(p.X)
    Xb = bf16_round(Xw)
    Xd = dev(Xb.astype(np.float32), torch.bfloat16)
    W0 = p.W0.astype(np.float32)
    # the rows the first pass starts from: W0 normalised in FP64, stored FP32
    W064 = W0.astype(np.float64)
    B = (W064 / np.linalg.norm(W064, axis=1, keepdims=True)).astype(np.float32).astype(np.float64)
    Bp = bf16_round(B)
    fp = ctx.fixed_point(Xd, dev(W0), Xw_f32=dev(Xb.astype(np.float32)), max_iter=1, tol=1e-6,
                         precision="bf16", tol_bf16=1e-5, refine_iters=0, check_every=1,
                         refine_groups=False, bf16_row_terms=1)
    W1 = fp["W"].cpu().numpy().astype(np.float64)
    assert fp["thread_iters"] == K
    # the single-update entry point on the rounded rows (lo part zero)
    G, _ = ctx.update(Xd, dev(Bp.astype(np.float32)))
    G = G.cpu().numpy()
    Gn = G / np.linalg.norm(G, axis=1, keepdims=True)
    sgn = np.sign(np.sum(Gn * W1, axis=1, keepdims=True))
    assert np.max(np.abs(W1 - sgn * Gn)) <= 2e-6
    # the oracle's update of the rounded rows; the kernel rounds z^3 to BF16
    Gr, _ = ica.update(Xb, Bp)
    Z = Bp @ Xb
    bound = 2.0 ** -9 * (np.abs(Z) ** 3 @ np.abs(Xb).T) / T + 2e-5 + 1e-5 * np.abs(Gr)
    assert np.all(np.abs(G - Gr) <= bound)
    Grn = Gr / np.linalg.norm(Gr, axis=1, keepdims=True)
    tol_rows = 2.0 * np.linalg.norm(bound, axis=1) / np.linalg.norm(Gr, axis=1) + 2e-6
    assert np.all(np.linalg.norm(W1 - sgn * Grn, axis=1) <= tol_rows)
    # with the linear term on the unrounded row the pass would land elsewhere
    Gx = G - 3.0 * (B - Bp)
    Gxn = Gx / np.linalg.norm(Gx, axis=1, keepdims=True)
    assert np.median(np.linalg.norm(W1 - sgn * Gxn, axis=1)) > 50 * 2e-6


@pytest.mark.parametrize("form,tol_bf16", [(0, 1e-3), (1, 1e-5), (2, 1e-5), (3, 1e-5), (2, 1e-3),
                                           (4, 1e-3)])
def test_row_forms_match_oracle_eeg_shaped(form, tol_bf16):
    from paper_2408_17118_amd import oica
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "eeg_shaped_n64_oracle.json")))
    p = synth.eeg_shaped()
    c = oica.Context(0)
    res = oica.ordering_ica(c, dev(p.X), dev(p.W0.astype(np.float32)), tol=1e-6, max_iter=1000,
                            precision="bf16", tol_bf16=tol_bf16, refine_iters=5, bf16_row_terms=form)
    print(f"form {form}, tol_bf16 {tol_bf16}: passes {res['fp']['passes']}, "
          f"thread-iterations {res['fp']['thread_iters']}, "
          f"refinement {res['fp']['refine_thread_iters']}")
    assert res["n_unique"] == ref["n_unique"]
    _check_against(res, np.array(ref["U_raw"]), np.array(ref["alpha"]), np.array(ref["upsilon"]),
                   ref["n_accepted"], f"form {form}")
    c.close()
