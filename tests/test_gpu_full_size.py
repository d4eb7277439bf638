"""The irregular and the K = 32 workloads at their full sizes, in the launch
configuration the benchmark times, against the FP64 oracle.

* Erdos-Renyi, 200,000 binary variables, average degree 6, C = 2.5 (RnBP
  p = 0.3 against LBP): one LBP sweep over every message, and three RnBP
  iterations with dynamic p, each checked as one step of Alg. 1.
* Potts grid 500 x 500, K = 32, one shared table exp(beta [x_i = x_j]) with
  per-edge scales (the matrix-core kernel): one sweep over every message with
  FP32 operands (1e-6 relative) and with BF16 operands (2^-7, the BF16
  product's bound), and three RnBP iterations with dynamic p, which read and
  write rows with outcome flags.

Bars and the band rule as in the multi-iteration tests: frontier equal except
for messages whose FP64 residual lies within 1e-6 of eps.
"""
import numpy as np
import pytest

import oracle
from paper_1909_11469_amd import inputs
from test_gpu_multi_iteration import _check_iteration, _random_rows

pytestmark = pytest.mark.gpu

SWEEP_TOL = 1e-6
BF16_SWEEP = 2.0 ** -7


@pytest.fixture(scope="module")
def bp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1909_11469_amd import bp as mod
    return mod


def _sweep(bp, prob, S, flags=0):
    with bp.Graph(prob, flags=flags) as g:
        g.set_state(S, t=0)
        start, _ = g.get_state()
        g.run("lbp", eps=0.0, max_iters=1, warm_start=True)
        m, _ = g.get_state()
    cand, _ = oracle.evaluate(prob, start.astype(np.float64))
    return np.max(np.abs(m - cand) / np.max(np.abs(cand), axis=1, keepdims=True), axis=1)


def _prefix_runs(bp, prob, S0, t0, kmax, p, seed, eps, flags=0):
    out = []
    with bp.Graph(prob, flags=flags) as g:
        for k in range(kmax + 1):
            g.set_state(S0, t=t0, prev_active=-1)
            r = g.run("rnbp", eps=eps, p=p, seed=seed, max_iters=k, warm_start=True,
                      check_every=16)
            m, st = g.get_state()
            out.append((m, st, r))
    return out


@pytest.fixture(scope="module")
def er200k():
    return inputs.er_graph(200000, 6.0, 2.5, 0)


@pytest.fixture(scope="module")
def potts500():
    return inputs.potts_grid(500, 500, 32, 1.0, 0)


def test_er_200k_single_sweep_full_size(bp, er200k):
    E = 2 * len(er200k["edges"])
    S = _random_rows(E, 2, 3, 0.05)
    err = _sweep(bp, er200k, S)
    print(f"ER 200k: {E} messages, max rel err {err.max():.2e}")
    assert err.max() <= SWEEP_TOL


def test_er_200k_rnbp_dynamic_p_three_iterations(bp, er200k):
    E = 2 * len(er200k["edges"])
    S0 = _random_rows(E, 2, 4, 0.3)
    p, seed, eps, t0, kmax = 0.3, 6, 1e-4, 4, 3
    runs = _prefix_runs(bp, er200k, S0, t0, kmax, p, seed, eps)
    for k in range(1, kmax + 1):
        assert runs[k][2]["iterations"] == k
        _check_iteration(er200k, runs[k - 1], runs[k], runs[k][2], "rnbp", p, seed, eps, True,
                         max_band=E // 10000)


def test_potts_500_single_sweep_full_size(bp, potts500):
    E = 2 * len(potts500["edges"])
    S = _random_rows(E, 32, 5, 0.2)
    err = _sweep(bp, potts500, S)
    err16 = _sweep(bp, potts500, S, flags=16)
    print(f"Potts 500x500 K=32: {E} messages, max rel err FP32 {err.max():.2e}, "
          f"BF16 {err16.max():.2e}")
    assert err.max() <= SWEEP_TOL
    assert err16.max() <= BF16_SWEEP


def test_potts_500_rnbp_dynamic_p_three_iterations(bp, potts500):
    E = 2 * len(potts500["edges"])
    S0 = _random_rows(E, 32, 6, 0.3)
    p, seed, eps, t0, kmax = 0.5, 2, 1e-3, 3, 3
    runs = _prefix_runs(bp, potts500, S0, t0, kmax, p, seed, eps)
    for k in range(1, kmax + 1):
        assert runs[k][2]["iterations"] == k
        # about 1e-4 of the messages have an FP64 residual within 1e-6 of eps
        _check_iteration(potts500, runs[k - 1], runs[k], runs[k][2], "rnbp", p, seed, eps, True,
                         max_band=E // 2000)
    for m, _, _ in runs:
        assert np.all(m >= 0.0)
