"""K = 32 Potts with BF16 operands on the matrix cores (BP_FLAG_BF16_MATRIX_CORES)
against the FP64 oracle: the error the reduced-precision product costs.

The product of Eq. (2), c(y) = sum_x P[x][y] g(x), takes g and P rounded to
BF16 (8-bit mantissas, round to nearest even: relative error <= 2^-9 each) and
accumulates in FP32.  Every term is positive, so c carries a relative error of
at most about 2^-8; after normalisation an entry of the message is off by at
most about 2 * 2^-8 = 2^-7 relative to the largest entry.  That is the bar of
the one-sweep test (far above the 1e-6 of the FP32 paths); converged beliefs
on a unique-fixed-point problem are held to 1e-2.  The measured errors are
printed.
"""
import numpy as np
import pytest

import oracle
from paper_1909_11469_amd import inputs

pytestmark = pytest.mark.gpu

BF16_SWEEP = 2.0 ** -7


@pytest.fixture(scope="module")
def bp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1909_11469_amd import bp as mod
    return mod


def _random_state(E, K, seed):
    m = np.random.default_rng(seed).uniform(0.2, 1.0, size=(E, K))
    m /= m.sum(1, keepdims=True)
    return m.astype(np.float32)


@pytest.mark.parametrize("side", [12, 37])
def test_bf16_single_sweep_error(bp, side):
    prob = inputs.potts_grid(side, side + 3, 32, 1.0, 1)
    E = 2 * len(prob["edges"])
    S = _random_state(E, 32, 2)
    out = {}
    for name, flags in (("fp32", 0), ("bf16", bp.BP_FLAG_BF16_MATRIX_CORES)):
        with bp.Graph(prob, flags=flags) as g:
            g.set_state(S, t=0)
            start, _ = g.get_state()
            g.run("lbp", eps=0.0, max_iters=1, warm_start=True)
            out[name], _ = g.get_state()
    cand, _ = oracle.evaluate(prob, start.astype(np.float64))
    rel = {k: np.max(np.abs(v - cand) / np.max(cand, axis=1, keepdims=True)) for k, v in out.items()}
    print(f"potts {side}x{side + 3} K=32 one sweep, max rel error vs FP64: "
          f"fp32 {rel['fp32']:.2e}, bf16 {rel['bf16']:.2e}")
    assert rel["fp32"] <= 1e-6
    assert 0.0 < rel["bf16"] <= BF16_SWEEP


def test_bf16_converged_marginals_error(bp):
    prob = inputs.potts_grid(12, 12, 32, 1.0, 0)
    ref = oracle.run(prob, oracle.LBP, eps=1e-6, max_iters=10000)
    assert ref["converged"]
    with bp.Graph(prob, flags=bp.BP_FLAG_BF16_MATRIX_CORES) as g:
        r = g.run("rnbp", eps=1e-5, p=0.5, seed=3, max_iters=100000)
        marg = g.marginals()
    assert r["converged"]
    err = float(np.max(np.abs(marg - ref["marginals"])))
    print(f"potts 12x12 K=32 bf16: max|marginal - oracle| = {err:.3e}")
    assert err <= 1e-2
