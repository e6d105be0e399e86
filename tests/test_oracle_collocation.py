"""Pins of the collocation part of the oracle (Section 4)."""
import itertools
import json
import os
from math import prod

import numpy as np
import pytest

from oracle.collocation import Grid, gauss_hermite
from workloads import problem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def dfact(n):
    return prod(range(n, 0, -2)) if n > 0 else 1


def normal_moment(k):
    return 0.0 if k % 2 else float(dfact(k - 1))


def test_gauss_hermite_textbook_rules():
    gold = json.load(open(os.path.join(GOLD, "gauss_hermite.json")))["rules"]
    for m, r in gold.items():
        x, w = gauss_hermite(int(m))
        assert np.allclose(x, r["x"], atol=1e-15)
        assert np.allclose(w, r["w"], atol=1e-15)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 7, 15])
def test_gauss_hermite_exact_to_degree_2m_minus_1(m):
    x, w = gauss_hermite(m)
    for k in range(2 * m):
        scale = w @ np.abs(x) ** k
        assert abs(w @ x ** k - normal_moment(k)) < 1e-13 * scale + 1e-14
    # and not exact at degree 2m
    assert abs(w @ x ** (2 * m) - normal_moment(2 * m)) > 1e-6


def _regions(nterms):
    return [{"nterm": n} for n in nterms]


def test_tensor_grid_counts_and_exactness():
    gold = json.load(open(os.path.join(GOLD, "paper_counts.json")))["grid_sizes"]
    for m, N, n in gold["tensor"]:
        assert m ** N == n
    g = Grid(_regions([1, 2]), {"kind": "tensor", "m": 3})
    assert g.nreal == 27 and abs(g.weights.sum() - 1) < 1e-15
    # per-dimension degree 2m-1 = 5
    for ks in itertools.product(range(6), repeat=3):
        val = np.sum(g.weights * np.prod(g.points ** np.array(ks), axis=1))
        assert abs(val - prod(normal_moment(k) for k in ks)) < 1e-12 * max(1, prod(normal_moment(k) for k in ks))
    # last dimension fastest
    assert list(g.ids[1]) == [0, 0, 1]


def test_sparse_grid_level1_count_is_2N_plus_1():
    gold = json.load(open(os.path.join(GOLD, "paper_counts.json")))["grid_sizes"]
    for N, n in gold["sparse_level1"]:
        g = Grid(_regions([N]), {"kind": "sparse", "level": 1, "growth": "paper"})
        assert g.nreal == n


@pytest.mark.parametrize("N,level", [(2, 2), (3, 2), (4, 1), (3, 3)])
def test_sparse_grid_exact_to_total_degree(N, level):
    g = Grid(_regions([N]), {"kind": "sparse", "level": level, "growth": "paper"})
    assert abs(g.weights.sum() - 1.0) < 1e-13
    D = 2 * level + 1
    for ks in itertools.product(range(D + 1), repeat=N):
        if sum(ks) > D:
            continue
        val = np.sum(g.weights * np.prod(g.points ** np.array(ks), axis=1))
        ex = prod(normal_moment(k) for k in ks)
        assert abs(val - ex) < 1e-10 * max(1.0, ex), (ks, val, ex)


def test_sparse_grid_cfg1_exactness_and_negative_weights():
    p = problem("cfg1")
    g = Grid(p["regions"], p["rule"])
    assert g.nreal == 361 and g.nlocal == [37, 37, 37, 37]
    assert (g.weights < 0).sum() > 0
    rng = np.random.default_rng(0)
    for _ in range(40):
        ks = np.zeros(12, dtype=int)
        deg = int(rng.integers(0, 6))
        for _ in range(deg):
            ks[rng.integers(0, 12)] += 1
        val = np.sum(g.weights * np.prod(g.points ** ks, axis=1))
        ex = prod(normal_moment(int(k)) for k in ks)
        assert abs(val - ex) < 1e-10 * max(1.0, ex)


def test_local_index_table_is_consistent():
    for name in ("cfg0", "cfg1", "cfg2"):
        p = problem(name)
        g = Grid(p["regions"], p["rule"])
        for r in range(len(p["regions"])):
            lp = g.local_points(r)
            o = g.dim_off
            assert np.array_equal(lp[g.g2l[:, r]], g.points[:, o[r]:o[r + 1]])
            # local points are sorted lexicographically by node ids
            ids = g.local_ids[r]
            assert all(tuple(ids[k]) < tuple(ids[k + 1]) for k in range(ids.shape[0] - 1))


def test_local_set_sizes_against_paper_ratios():
    """Tensor: N_real(j) = m^N_term(j); level-1 sparse: 2 N_term(j) + 1 (Section 6)."""
    g = Grid(_regions([2, 9]), {"kind": "tensor", "m": 2})
    assert g.nreal == 2048 and g.nlocal == [4, 512]
    g = Grid(_regions([25, 25]), {"kind": "sparse", "level": 1, "growth": "paper"})
    assert g.nreal == 101 and g.nlocal == [51, 51]
    g = Grid(_regions([196, 4]), {"kind": "sparse", "level": 1, "growth": "paper"})
    assert g.nreal == 401 and g.nlocal == [393, 9]
