"""Pins of the oracle's tree: clusters, BFS serial order and the RKV filter.

Sec. 3.1 (eqs. 1-2) and Sec. 3.4 (BFS linearisation); readings C2-C4.
* hand-derived BFS tables for two small grids;
* an independent brute-force BFS over an explicitly built tree;
* the filter on constant views against numpy's weighted average with the
  binomial weights, rounded half up with exact fractions.
"""
from collections import deque
from fractions import Fraction
from math import comb, floor

import numpy as np
import pytest

import oracle


def test_bfs_hand_derived_two_levels():
    # 4x2 grid, cluster 2: top nodes (0,0), (1,0); children row-major in cluster
    p = oracle.Params(4, 2, 4, 4, 4, 2, (2,))
    path, root = oracle.tree_tables(p)
    assert list(path[:, 0]) == [0, 1, 4, 5, 2, 3, 6, 7]
    assert list(root) == [0, 0, 1, 1, 0, 0, 1, 1]


def test_bfs_hand_derived_three_levels():
    # 4x4 grid, clusters (2,2): level 1 is 2x2, one top node
    p = oracle.Params(4, 4, 4, 4, 4, 3, (2, 2))
    path, root = oracle.tree_tables(p)
    assert list(path[:, 1]) == [0, 0, 1, 1, 0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 3, 3]
    assert list(path[:, 0]) == [4, 5, 8, 9, 6, 7, 10, 11, 12, 13, 16, 17, 14, 15, 18, 19]
    assert list(root) == [0] * 16


def brute_tree(U, V, clusters):
    """Explicit tree: level-l nodes as (l, x, y); children listed by scanning
    every node of the level below and keeping those inside the cluster."""
    grids = [(U, V)]
    for c in clusters:
        pu, pv = grids[-1]
        grids.append((-(-pu // c), -(-pv // c)))
    L = len(grids)
    children = {}
    for l in range(1, L):
        c = clusters[l - 1]
        cu, cv = grids[l - 1]
        for y in range(grids[l][1]):
            for x in range(grids[l][0]):
                kids = [(l - 1, xx, yy) for yy in range(cv) for xx in range(cu)
                        if x * c <= xx < (x + 1) * c and y * c <= yy < (y + 1) * c]
                children[(l, x, y)] = kids
    order = []
    queue = deque((L - 1, x, y) for y in range(grids[-1][1]) for x in range(grids[-1][0]))
    while queue:
        n = queue.popleft()
        order.append(n)
        queue.extend(children.get(n, []))
    srv = {}
    for n in order:
        if n[0] < L - 1:
            srv[n] = len(srv)
    return grids, children, srv


@pytest.mark.parametrize("U,V,clusters", [
    (8, 8, (2,)), (17, 17, (2, 3)), (9, 9, (2, 2)), (3, 5, (2,)), (5, 3, (3,)),
    (7, 4, (2, 2, 2)), (17, 17, (2, 2, 2, 2)), (1, 1, ()), (6, 1, (4,)),
])
def test_bfs_matches_brute_force(U, V, clusters):
    L = len(clusters) + 1
    p = oracle.Params(U, V, 4, 4, 4, L, tuple(clusters))
    path, root = oracle.tree_tables(p)
    grids, children, srv = brute_tree(U, V, clusters)
    parent = {k: n for n, ks in children.items() for k in ks}
    assert oracle.geometry(p).n_srv == len(srv)
    for vi in range(U * V):
        node = (0, vi % U, vi // U)
        for l in range(L - 1):
            assert path[vi, l] == srv[node]
            node = parent[node]
        assert root[vi] == node[2] * grids[-1][0] + node[1]


def _constant_views(U, V, vals, W=4, H=4):
    lf = np.zeros((V, U, H, W, 3), dtype=np.uint8)
    for vi, a in enumerate(vals):
        lf[vi // U, vi % U] = a
    return lf


@pytest.mark.parametrize("U,V,c", [(4, 4, 2), (6, 6, 3), (5, 4, 3), (3, 3, 2), (8, 3, 4), (17, 17, 3)])
def test_filter_is_rounded_binomial_mean(U, V, c):
    rng = np.random.default_rng(U * 100 + V * 10 + c)
    vals = rng.integers(0, 256, U * V)
    lf = _constant_views(U, V, vals)
    # grey views: Y = value, Co = Cg = 0
    p = oracle.Params(U, V, 4, 4, 4, 2, (c,))
    levels = oracle.rkv_tree(lf, p)
    top = levels[1]
    for y in range(top.shape[0]):
        for x in range(top.shape[1]):
            members, weights = [], []
            for yy in range(y * c, min((y + 1) * c, V)):
                for xx in range(x * c, min((x + 1) * c, U)):
                    members.append(int(vals[yy * U + xx]))
                    weights.append(comb(c - 1, xx - x * c) * comb(c - 1, yy - y * c))
            mean = Fraction(int(np.dot(members, weights)), int(np.sum(weights)))
            assert abs(float(mean) - np.average(members, weights=weights)) < 1e-9
            expect = floor(mean + Fraction(1, 2))
            assert np.all(top[y, x, 0] == expect), (x, y)
            assert np.all(top[y, x, 1:] == 0)


def test_filter_negative_chroma_rounds_half_up():
    # Co = R - B: views with Co = -3 and -4 average to -3.5 -> -3 (half up)
    lf = np.zeros((1, 2, 4, 4, 3), dtype=np.uint8)
    lf[0, 0] = (10, 10, 13)
    lf[0, 1] = (10, 10, 14)
    levels = oracle.rkv_tree(lf, oracle.Params(2, 1, 4, 4, 4, 2, (2,)))
    assert np.all(levels[1][0, 0, 1] == -3)


def test_constant_light_field_is_fixed_point():
    lf = np.full((9, 9, 8, 8, 3), 77, dtype=np.uint8)
    lf[..., 0] = 120
    p = oracle.Params(9, 9, 8, 8, 4, 3, (2, 2))
    levels = oracle.rkv_tree(lf, p)
    for l in range(1, 3):
        assert np.array_equal(levels[l][0, 0], levels[0][0, 0])
        assert np.all(levels[l] == levels[0][0, 0][None, None])
