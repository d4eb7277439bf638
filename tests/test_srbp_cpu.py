"""The serial residual BP baseline (libsrbp, include/srbp.h) on the CPU, against
the FP64 oracle's serial residual BP (itself pinned in test_oracle_pins.py).

Both compute every candidate with the literal product of Eq. (2) in the same
factor order and pick the largest residual with the same tie rule, so the
commit sequence is expected to be identical and the messages equal bit for bit;
the tests assert the sequence exactly and the values within 1e-13.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1909_11469_amd import inputs
from tests import exact_refs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def srbp():
    from paper_1909_11469_amd import srbp as mod
    return mod


def test_header_declarations_exported(srbp):
    text = open(os.path.join(ROOT, "include", "srbp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    declared = sorted(set(re.findall(r"\b(srbp_\w+)\s*\(", text)))
    assert declared == sorted(srbp.EXPORTED)
    raw = ctypes.CDLL(srbp.LIB_PATH)
    for name in declared:
        assert hasattr(raw, name), name


def test_stats_layout_matches_header(srbp, tmp_path):
    import subprocess
    S = srbp.srbp_stats
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "srbp.h"', "int main(void) {",
             'printf("size %zu\\n", sizeof(srbp_stats));']
    lines += [f'printf("{f} %zu\\n", offsetof(srbp_stats, {f}));' for f, _ in S._fields_]
    lines.append("return 0; }")
    src = tmp_path / "l.c"
    src.write_text("\n".join(lines))
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(tmp_path / "l")], check=True)
    out = dict(l.split() for l in subprocess.run([str(tmp_path / "l")], capture_output=True,
                                                 text=True).stdout.splitlines())
    assert int(out["size"]) == ctypes.sizeof(S)
    for f, _ in S._fields_:
        assert int(out[f]) == getattr(S, f).offset, f


PROBLEMS = {
    "ising_C1": lambda: inputs.ising_grid(10, 10, 1.0, 0),
    "ising_C2.5": lambda: inputs.ising_grid(8, 9, 2.5, 1),
    "paper_ising": lambda: inputs.paper_ising_grid(9, 9, 2.5, 2),
    "tree_K3": lambda: inputs.random_tree(30, 3, 1),
    "shared_K4": lambda: inputs.shared_table_graph(20, 40, 4, 3),
    "dense_K3": lambda: inputs.random_dense_graph(15, 30, 3, 2),
    "er": lambda: inputs.er_graph(60, 5.0, 1.5, 4),
    "potts_K5": lambda: inputs.potts_grid(5, 6, 5, 1.0, 5),
}


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_sequence_and_messages_equal_oracle(srbp, name):
    prob = PROBLEMS[name]()
    cap = 20000
    a = srbp.srbp_solve(prob, eps=1e-6, max_updates=cap, msgs=True, trace_len=cap)
    b = oracle.srbp(prob, eps=1e-6, max_updates=cap, trace=True)
    assert a["converged"] == b["converged"] and a["updates"] == b["updates"]
    np.testing.assert_array_equal(a["trace"], b["trace"])
    np.testing.assert_allclose(a["msgs"], b["msgs"], atol=1e-13, rtol=0)
    np.testing.assert_allclose(a["marginals"], b["marginals"], atol=1e-13, rtol=0)
    if a["converged"]:
        assert a["max_residual"] <= 1e-6
    # every update re-evaluates only the messages that read the committed one
    assert a["evaluations"] < 2 * len(prob["edges"]) + a["updates"] * 64


def test_tree_exact_and_high_degree_star(srbp):
    prob = inputs.random_tree(11, 3, 7)
    r = srbp.srbp_solve(prob, eps=1e-14)
    assert r["converged"]
    np.testing.assert_allclose(r["marginals"], exact_refs.brute_force_marginals(prob), atol=1e-11)
    # 1100 leaves: the centre's products pass 2^-1100 and are rescaled
    # (each leaf commit re-evaluates every centre -> leaf message, O(deg^2))
    n = 1101
    rng = np.random.default_rng(3)
    edges = np.array([(0, i) for i in range(1, n)], np.int32)
    star = dict(N=n, K=2, edges=edges, log_unary=rng.normal(size=(n, 2)),
                pair_kind=inputs.PAIR_ISING, coupling=rng.uniform(-1, 1, n - 1))
    r = srbp.srbp_solve(star, eps=1e-13)
    assert r["converged"]
    np.testing.assert_allclose(r["marginals"], exact_refs.star_marginals(star), atol=1e-10)


def test_caps_and_degenerate_inputs(srbp):
    prob = inputs.ising_grid(12, 12, 3.0, 9)
    r = srbp.srbp_solve(prob, eps=1e-12, max_updates=500)
    assert not r["converged"] and r["updates"] == 500
    r = srbp.srbp_solve(inputs.paper_ising_grid(60, 60, 8.0, 1), eps=1e-12, time_limit_s=0.05)
    assert r["timed_out"] and not r["converged"] and r["seconds"] < 5
    # no edges: converged at once, beliefs are the normalised unaries
    lu = np.array([[0.0, 1.0], [2.0, -1.0]])
    iso = dict(N=2, K=2, edges=np.zeros((0, 2), np.int32), log_unary=lu,
               pair_kind=inputs.PAIR_ISING, coupling=np.zeros(0))
    r = srbp.srbp_solve(iso)
    assert r["converged"] and r["updates"] == 0
    np.testing.assert_allclose(r["marginals"], np.exp(lu) / np.exp(lu).sum(1, keepdims=True))


def test_rejects_invalid(srbp):
    from paper_1909_11469_amd import bp
    prob = inputs.ising_grid(3, 3, 1.0, 0)
    for bad in (dict(edges=np.array([[0, 0]], np.int32), coupling=np.zeros(1)),
                dict(edges=np.array([[0, 9]], np.int32), coupling=np.zeros(1)),
                dict(edges=np.array([[0, 1], [1, 0]], np.int32), coupling=np.zeros(2))):
        with pytest.raises(bp.BpError):
            srbp.srbp_solve({**prob, **bad})
    with pytest.raises(bp.BpError):
        srbp.srbp_solve(prob, eps=-1.0)
