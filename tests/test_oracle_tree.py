"""Pins of the oracle's region tree, levels and prolongations (Section 3.1, 3.2).

Checked against: the paper's worked example (structure printed in Section 3.1.1
Steps 2-4 and Section 3.1.2; coordinates chosen to reproduce its insertion
history), a literal sequential-insertion tree written here (brute force), the
corrected depth bound of Theorem 1, partition of unity and multilinear
reproduction of the interpolation, and Theorem 2 (capacity 9 on a uniform grid
gives the classical geometric-multigrid bilinear prolongation).
"""
import json
import os

import numpy as np
import pytest

from oracle import tree

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# literal sequential insertion (Section 3.1.1 Step 2), written independently:
# points are inserted one by one; a leaf that exceeds the capacity is split at
# its midlines (upper child iff x >= mid) and hands its points to the children.
# ---------------------------------------------------------------------------
def sequential_tree(coords, cap):
    m, M = float(coords.min()), float(coords.max())
    d = coords.shape[1]
    leaves = {(1, (0,) * d): []}
    internal_nodes = set()

    def mid_of(lo, depth):
        half = 1 << (48 - depth - 1)
        mid = [m + (M - m) * ((lo[a] + half) * 2.0 ** -47) for a in range(d)]
        return mid, half

    def descend(p, node):
        depth, lo = node
        mid, half = mid_of(lo, depth)
        clo = tuple(lo[a] + (half if coords[p, a] >= mid[a] else 0) for a in range(d))
        return (depth + 1, clo)

    def insert(p, node):
        while node in internal_nodes:
            node = descend(p, node)
        leaves.setdefault(node, []).append(p)
        if len(leaves[node]) > cap:
            if node[0] >= 48:
                raise ValueError("depth limit")
            pts = leaves.pop(node)
            internal_nodes.add(node)
            for q in pts:
                insert(q, node)

    for p in range(coords.shape[0]):
        insert(p, (1, (0,) * d))
    out_depth = np.zeros(coords.shape[0], dtype=np.int64)
    out_lo = np.zeros((coords.shape[0], d), dtype=np.int64)
    for (depth, lo), pts in leaves.items():
        for q in pts:
            out_depth[q] = depth
            out_lo[q] = lo
    return out_depth, out_lo


def _clouds():
    rng = np.random.default_rng(7)
    yield rng.uniform(0, 1, (300, 2)), 4
    yield rng.uniform(-3, 5, (400, 3)), 8
    c = np.concatenate([rng.normal(0, 0.01, (150, 2)), rng.uniform(0, 1, (100, 2))])
    yield c, 4
    g = np.stack(np.meshgrid(np.linspace(0, 1, 9), np.linspace(0, 1, 9)), -1).reshape(-1, 2)
    yield g, 4
    yield g, 9
    yield rng.uniform(0, 1, (200, 3)) ** 3, 3


@pytest.mark.parametrize("case", range(6))
def test_tree_matches_sequential_insertion(case):
    coords, cap = list(_clouds())[case]
    dep, lo = tree.build_tree(coords, cap)
    dep2, lo2 = sequential_tree(coords, cap)
    assert np.array_equal(dep, dep2)
    assert np.array_equal(lo, lo2)


@pytest.mark.parametrize("case", range(6))
def test_tree_capacity_invariants_and_depth_bound(case):
    coords, cap = list(_clouds())[case]
    dep, lo = tree.build_tree(coords, cap)
    N, d = coords.shape
    leaves = {}
    for i in range(N):
        leaves.setdefault((int(dep[i]), tuple(lo[i])), []).append(i)
    for (D, L), pts in leaves.items():
        assert len(pts) <= cap                          # leaves hold at most cap
        if D > 1:                                       # the parent held more than cap
            ps = 1 << (48 - (D - 1))
            plo = np.array(L) // ps * ps
            inside = np.all(lo // ps * ps == plo, axis=1) & (dep >= D)
            assert inside.sum() > cap
    # depth <= 2 + log2(diam(D1)/d_min)   (Theorem 1, bound taken over internal nodes)
    from scipy.spatial.distance import pdist
    dmin = pdist(coords).min()
    m, M = coords.min(), coords.max()
    diam = np.sqrt(d) * (M - m)
    assert dep.max() <= 2 + np.log2(diam / dmin)


def test_duplicate_vertices_hit_the_depth_limit():
    c = np.array([[0.0, 0.0], [1.0, 1.0], [0.5, 0.5], [0.5, 0.5], [0.5, 0.5]])
    with pytest.raises(ValueError):
        tree.build_tree(c, 2)


def test_worked_example_of_the_paper():
    g = json.load(open(os.path.join(GOLD, "worked_example_2d.json")))
    coords = np.array(g["coords"], dtype=np.float64)
    cap = g["capacity"]
    dep, lo = tree.build_tree(coords, cap)
    assert dep.max() == g["tree_height"]
    # leaf membership as printed (1-based vertex numbers)
    groups = {}
    for i in range(coords.shape[0]):
        groups.setdefault((int(dep[i]), tuple(lo[i])), set()).add(i + 1)
    expected = {frozenset(v) for v in g["leaves"].values()}
    assert {frozenset(v) for v in groups.values()} == expected
    for name, members in g["leaves"].items():
        i = members[0] - 1
        assert dep[i] == g["leaf_depth"][name]
    lv = tree.build_levels(coords, coords, np.arange(coords.shape[0]), cap)
    # the boundary vertices 9 and 19 give zero weight to some corners, but the
    # level-1 vertex set is the set of all leaf corners (17 of them)
    nonempty = tree.corners(*lv.regions[0][::1])
    allc = np.unique(lv.codec.encode(nonempty.reshape(-1, 2)))
    assert allc.size == g["n_coarse_vertices_level1"]
    assert lv.level_codes[0].size <= allc.size
    assert len(lv.level_codes) == 3
    assert lv.level_codes[1].size == g["n_vertices_level2"]
    assert lv.level_codes[2].size == g["n_vertices_level3"]
    # every nonzero weight of a fine vertex sits on a corner of its own leaf
    P0 = lv.prolong[0].tocoo()
    k1 = lv.level_keys(1)
    side = tree.side_of(dep)
    for r, c in zip(P0.row, P0.col):
        rel = k1[c] - lo[r]
        assert np.all((rel == 0) | (rel == side[r]))


def _grid(n, d):
    ax = np.linspace(0.0, 1.0, n)
    g = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), -1).reshape(-1, d)
    return g[:, ::-1].copy()      # x fastest


@pytest.mark.parametrize("d,n,cap", [(2, 9, 4), (2, 17, 4), (3, 5, 8)])
def test_partition_of_unity_and_multilinear_reproduction(d, n, cap):
    rng = np.random.default_rng(3)
    c = _grid(n, d)
    h = 1.0 / (n - 1)
    interior = np.all((c > 0) & (c < 1), axis=1)
    c[interior] += rng.uniform(-0.2 * h, 0.2 * h, (interior.sum(), d))
    free = np.flatnonzero(interior)
    pos = np.full(c.shape[0], -1)
    pos[np.arange(c.shape[0])] = np.arange(c.shape[0])
    lv = tree.build_levels(c, c[free], pos[free], cap)

    def g(x):           # a multilinear function
        out = 0.3 + 1.7 * x[:, 0] - 0.4 * x[:, 1] + 2.1 * x[:, 0] * x[:, 1]
        if d == 3:
            out = out + 0.9 * x[:, 2] - 1.3 * x[:, 0] * x[:, 2] + 0.7 * x[:, 0] * x[:, 1] * x[:, 2]
        return out
    fine = c[free]
    for l, P in enumerate(lv.prolong):
        rows = np.asarray(P.sum(axis=1)).ravel()
        assert np.allclose(rows, 1.0, atol=1e-14, rtol=0)
        coarse = lv.level_coords(l + 1)
        here = fine if l == 0 else lv.level_coords(l)
        assert np.allclose(P @ g(coarse), g(here), atol=1e-13, rtol=0)
        if l > 0:                       # lattice levels: weights in {1, 1/2, 1/4, 1/8}
            assert set(np.unique(P.data)) <= {1.0, 0.5, 0.25, 0.125}
    # levels below the fine one = max depth; the root level holds 2^d vertices
    assert len(lv.level_codes) == lv.max_depth
    assert lv.level_codes[-1].size == 2 ** d


@pytest.mark.parametrize("k", [2, 3, 4])
def test_theorem2_capacity9_gives_geometric_multigrid(k):
    """Uniform (2^k+1)^2 grid, capacity 9, all vertices in the tree: the leaves are
    the 2h squares and P_0 is the classical bilinear prolongation (1, 1/2, 1/4)."""
    n = 2 ** k + 1
    c = _grid(n, 2)
    lv = tree.build_levels(c, c, np.arange(c.shape[0]), 9)
    coarse = lv.level_coords(1)
    nc = 2 ** (k - 1) + 1
    assert coarse.shape[0] == nc * nc
    H = 2.0 / (n - 1)
    ci = np.rint(coarse / H).astype(int)
    cidx = {(int(a), int(b)): t for t, (a, b) in enumerate(ci)}
    expected = np.zeros((n * n, nc * nc))
    for j in range(n):
        for i in range(n):
            r = i + n * j
            xs = [(i // 2, 1.0)] if i % 2 == 0 else [(i // 2, 0.5), (i // 2 + 1, 0.5)]
            ys = [(j // 2, 1.0)] if j % 2 == 0 else [(j // 2, 0.5), (j // 2 + 1, 0.5)]
            for (a, wa) in xs:
                for (b, wb) in ys:
                    expected[r, cidx[(a, b)]] += wa * wb
    assert np.array_equal(lv.prolong[0].toarray(), expected)


def test_injection_rows_are_unit_vectors():
    rng = np.random.default_rng(5)
    c = rng.uniform(0, 1, (500, 2))
    lv = tree.build_levels(c, c, np.arange(500), 4)
    for l in range(1, len(lv.prolong)):
        P = lv.prolong[l].tocsr()
        nxt = lv.level_codes[l]
        cur = lv.level_codes[l - 1]
        inj = np.isin(cur, nxt)
        for i in np.flatnonzero(inj):
            row = P.getrow(i)
            assert row.nnz == 1 and row.data[0] == 1.0
            assert nxt[row.indices[0]] == cur[i]
