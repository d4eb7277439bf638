"""Seeded generators: shapes, counts, determinism and value ranges."""
import numpy as np

from paper_1909_11469_amd import inputs


def test_ising_20x20_counts():
    p = inputs.ising_grid(20, 20, 2.5, 0)
    assert p["N"] == 400 and p["K"] == 2
    assert p["edges"].shape == (760, 2)  # 1520 directed messages
    assert np.all(np.abs(p["coupling"]) <= 2.5)
    assert np.all(np.abs(p["h"]) <= 1.0)
    np.testing.assert_array_equal(p["log_unary"][:, 1], -p["log_unary"][:, 0])


def test_grid_edge_order_fast_equals_reference():
    for H, W in [(1, 7), (3, 5), (9, 4), (70, 70)]:
        np.testing.assert_array_equal(inputs.grid_edges(H, W), inputs._grid_edges_fast(H, W))


def test_seeded_determinism():
    a = inputs.ising_grid(12, 13, 1.0, 42)
    b = inputs.ising_grid(12, 13, 1.0, 42)
    c = inputs.ising_grid(12, 13, 1.0, 43)
    assert np.array_equal(a["coupling"], b["coupling"])
    assert not np.array_equal(a["coupling"], c["coupling"])


def test_er_graph_simple_and_sized():
    p = inputs.er_graph(5000, 6.0, 2.5, 1)
    e = p["edges"].astype(np.int64)
    assert e.shape == (15000, 2)
    assert np.all(e[:, 0] != e[:, 1])
    key = np.minimum(e[:, 0], e[:, 1]) * p["N"] + np.maximum(e[:, 0], e[:, 1])
    assert len(np.unique(key)) == len(key)
    deg = np.bincount(e.ravel(), minlength=p["N"])
    assert abs(deg.mean() - 6.0) < 1e-9
    assert (deg == 0).sum() > 0  # isolated nodes exist at e^-6 * n ~ 12


def test_potts_shape():
    p = inputs.potts_grid(6, 5, 32, 1.0, 3)
    assert p["log_unary"].shape == (30, 32)
    assert p["shared"].shape == (32, 32)
    assert np.all((p["edge_scale"] >= 0.5) & (p["edge_scale"] <= 1.5))
    assert np.isclose(p["shared"][0, 0], np.e) and p["shared"][0, 1] == 1.0
