"""Auxiliary region-tree, coarse levels and prolongation weights (oracle).

Test infrastructure only (see the package header).

Follows Section 3.1.1 (Steps 1-4: root square, point insertion with splitting
above a capacity threshold, elimination of empty leaves, fine-to-coarse vertex
correspondence), Section 3.1.2 (coarser levels by merging the deepest regions
into their parents until only the root is left) and Section 3.2 (bilinear
prolongation weights, identical for every displacement component). 3D is the
octree analogue, as the paper states for its 2D presentation.

Readings of the paper taken here:
  * root box: one min and one max over all coordinates of all tree vertices,
    D1 = [m, M]^d (Step 1 takes the smaller of the x/y minima and the larger of
    the x/y maxima);
  * a node holding more than ``capacity`` vertices is split (Step 2; the paper
    uses 4 in 2D; 3D is unstated and defaults to 8); the final tree of a
    point-region tree does not depend on the insertion order, so the points are
    distributed top-down level by level;
  * a vertex goes to the upper child along an axis iff its coordinate is >= the
    node's midline;
  * node geometry lives on an integer lattice: a depth-i node (root depth 1) has
    side 2^(48-i) key units and the coordinate of key K is
    m + (M - m) * (K * 2^-47), so every midline and corner is reproducible
    bit for bit; depth 48 nodes cannot split (duplicate vertices);
  * the printed weight formula of Section 3.2 is garbled (it gives weight 0 to a
    coincident corner); it is read as standard bilinear/trilinear interpolation,
    w = prod_a (1 - |x_a - c_a| / (hi_a - lo_a)), which is what Theorem 2's
    reduction to geometric multigrid requires;
  * coarser levels (Section 3.1.2): all regions of the current maximum depth are
    replaced by their parents; a level vertex that is also a vertex of the next
    level is injected (weight 1), any other one is interpolated from the corners
    of its merged parent (weights 1, 1/2, 1/4, 1/8 on the lattice);
  * coarse vertices whose prolongation column is identically zero are dropped;
  * canonical vertex order on coarse levels is lexicographic in (z, y, x) keys.

Parity: the tree, level vertex sets and weights are pinned in
tests/test_oracle_tree.py (capacity invariants, brute-force sequential
insertion, depth bound, partition of unity, multilinear reproduction,
Theorem 2's geometric-multigrid weights). The paper's 19-vertex worked example
lost its coordinates with its figures and is parity unpinned.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

KEY_TOP = 47          # keys are integers in [0, 2^47]; the root (depth 1) has side 2^47
MAX_DEPTH = 48        # depth-48 nodes have side 1 and cannot be split
KEY_SCALE = 2.0 ** -KEY_TOP


def side_of(depth):
    """Side length in key units of a node at ``depth`` (root depth 1)."""
    return np.left_shift(np.int64(1), (MAX_DEPTH - np.asarray(depth, dtype=np.int64)))


def root_box(coords: np.ndarray):
    """Section 3.1.1 Step 1: the square/cube [m, M]^d covering all vertices."""
    return float(coords.min()), float(coords.max())


def key_coord(m: float, M: float, K) -> np.ndarray:
    """Coordinate of lattice key K (same formula in every implementation)."""
    K = np.asarray(K, dtype=np.int64).astype(np.float64)
    return m + (M - m) * (K * KEY_SCALE)


def build_tree(coords: np.ndarray, capacity: int):
    """Section 3.1.1 Step 2: split every node holding more than ``capacity`` vertices.

    Returns (leaf_depth [N], leaf_lo [N, d] int64): the leaf holding each vertex.
    """
    N, d = coords.shape
    m, M = root_box(coords)
    depth = np.zeros(N, dtype=np.int64)
    lo = np.zeros((N, d), dtype=np.int64)
    pending = np.arange(N)
    for D in range(1, MAX_DEPTH + 1):
        if pending.size == 0:
            break
        _, inv, cnt = np.unique(lo[pending], axis=0, return_inverse=True, return_counts=True)
        inv = inv.ravel()
        stays = cnt[inv] <= capacity
        depth[pending[stays]] = D
        pending = pending[~stays]
        if pending.size == 0:
            break
        if D == MAX_DEPTH:
            raise ValueError("region tree exceeds its depth limit (duplicate vertices?)")
        half = np.int64(1) << np.int64(MAX_DEPTH - D - 1)     # child side
        mid = key_coord(m, M, lo[pending] + half)
        upper = coords[pending] >= mid
        lo[pending] += upper.astype(np.int64) * half
    return depth, lo


def _corner_bits(d: int) -> np.ndarray:
    """[2^d, d] 0/1 corner patterns, bit a of the index selects the upper side on axis a."""
    b = np.arange(1 << d)
    return ((b[:, None] >> np.arange(d)[None, :]) & 1).astype(np.int64)


class KeyCodec:
    """Packs lattice keys into one int64 whose order is (z, y, x) lexicographic.

    All keys of the hierarchy are multiples of the finest leaf side
    2^(48-Dmax), so K >> (48-Dmax) fits in Dmax bits per axis.
    """

    def __init__(self, d: int, max_depth: int):
        self.d = d
        self.shift = MAX_DEPTH - max_depth
        self.bits = max_depth
        if d * self.bits > 62:
            raise NotImplementedError("oracle key packing needs d*depth <= 62")

    def encode(self, K: np.ndarray) -> np.ndarray:
        K = np.asarray(K, dtype=np.int64) >> np.int64(self.shift)
        code = np.zeros(K.shape[0], dtype=np.int64)
        for a in range(self.d):
            code |= K[:, a] << np.int64(a * self.bits)
        return code

    def decode(self, code: np.ndarray) -> np.ndarray:
        mask = (np.int64(1) << np.int64(self.bits)) - 1
        K = np.stack([(code >> np.int64(a * self.bits)) & mask for a in range(self.d)], axis=1)
        return K << np.int64(self.shift)


def corners(depth: np.ndarray, lo: np.ndarray) -> np.ndarray:
    """All 2^d corner keys of the given regions: [n_regions, 2^d, d]."""
    d = lo.shape[1]
    s = side_of(depth)
    return lo[:, None, :] + _corner_bits(d)[None, :, :] * s[:, None, None]


@dataclass
class TreeLevels:
    m: float
    M: float
    capacity: int
    max_depth: int
    codec: KeyCodec
    level_codes: list        # level l >= 1: sorted int64 codes of the active vertices
    prolong: list            # P_l (l >= 0): scalar CSR [n_l, n_{l+1}]
    regions: list            # level l >= 1: (depth [r], lo [r, d])

    def level_keys(self, l: int) -> np.ndarray:
        return self.codec.decode(self.level_codes[l - 1])

    def level_coords(self, l: int) -> np.ndarray:
        return key_coord(self.m, self.M, self.level_keys(l))


def _lookup(sorted_codes: np.ndarray, q: np.ndarray):
    pos = np.searchsorted(sorted_codes, q)
    pos_c = np.minimum(pos, sorted_codes.size - 1)
    found = (pos < sorted_codes.size) & (sorted_codes[pos_c] == q)
    return pos_c, found


def _drop_zero_columns(rows, cols_code, vals, n_rows):
    """Build P with columns = distinct column codes that carry a nonzero weight."""
    keep = vals != 0.0
    rows, cols_code, vals = rows[keep], cols_code[keep], vals[keep]
    codes, col = np.unique(cols_code, return_inverse=True)
    P = sp.csr_matrix((vals, (rows, col.ravel())), shape=(n_rows, codes.size))
    P.sum_duplicates()
    return P, codes


def build_levels(tree_coords: np.ndarray, fine_coords: np.ndarray, fine_in_tree: np.ndarray,
                 capacity: int) -> TreeLevels:
    """Region tree over ``tree_coords`` and the level hierarchy it defines.

    fine_coords: coordinates of the free fine vertices (rows of P_0), in the fine
    canonical order; fine_in_tree[i] is the index of fine vertex i among the tree
    vertices (every free vertex is a tree vertex).
    """
    N, d = tree_coords.shape
    m, M = root_box(tree_coords)
    leaf_depth, leaf_lo = build_tree(tree_coords, capacity)
    Dmax = int(leaf_depth.max())
    codec = KeyCodec(d, Dmax)
    bits = _corner_bits(d)

    # Step 3: the non-empty leaves form the first coarse level.
    reg = np.unique(np.concatenate([leaf_depth[:, None], leaf_lo], axis=1), axis=0)
    reg_depth, reg_lo = reg[:, 0], reg[:, 1:]

    # Step 4 + Section 3.2: P_0 row of each free fine vertex = multilinear weights
    # of its leaf's corners.
    fd = leaf_depth[fine_in_tree]
    flo = leaf_lo[fine_in_tree]
    fhi = flo + side_of(fd)[:, None]
    lo_c = key_coord(m, M, flo)
    hi_c = key_coord(m, M, fhi)
    t_up = (fine_coords - lo_c) / (hi_c - lo_c)
    t_dn = (hi_c - fine_coords) / (hi_c - lo_c)
    nf = fine_coords.shape[0]
    rows, ccode, vals = [], [], []
    for b in bits:
        w = np.ones(nf)
        for a in range(d):
            w = w * (t_up[:, a] if b[a] else t_dn[:, a])
        rows.append(np.arange(nf))
        ccode.append(codec.encode(flo + b[None, :] * side_of(fd)[:, None]))
        vals.append(w)
    P0, codes1 = _drop_zero_columns(np.concatenate(rows), np.concatenate(ccode),
                                    np.concatenate(vals), nf)
    prolong = [P0]
    level_codes = [codes1]
    regions = [(reg_depth, reg_lo)]

    # Section 3.1.2: merge the deepest regions until only the root is left.
    while not (reg_depth.size == 1 and reg_depth[0] == 1):
        Dstar = int(reg_depth.max())
        deep = reg_depth == Dstar
        ps = side_of(Dstar - 1)
        par_lo = (reg_lo[deep] // ps) * ps
        new = np.concatenate([
            np.concatenate([reg_depth[~deep, None], reg_lo[~deep]], axis=1),
            np.concatenate([np.full((par_lo.shape[0], 1), Dstar - 1), par_lo], axis=1),
        ])
        new = np.unique(new, axis=0)
        new_depth, new_lo = new[:, 0], new[:, 1:]
        next_codes = np.unique(codec.encode(corners(new_depth, new_lo).reshape(-1, d)))

        cur = level_codes[-1]
        n_cur = cur.size
        _, inj = _lookup(next_codes, cur)
        # parent of some merged region that has the vertex as a corner
        cc = corners(reg_depth[deep], reg_lo[deep])                 # [r, 2^d, d]
        c_code = codec.encode(cc.reshape(-1, d))
        c_par = np.repeat(par_lo, 1 << d, axis=0)
        order = np.argsort(c_code, kind="stable")
        c_code, c_par = c_code[order], c_par[order]
        rows, ccode, vals = [], [], []
        ir = np.flatnonzero(inj)
        rows.append(ir); ccode.append(cur[ir]); vals.append(np.ones(ir.size))
        it = np.flatnonzero(~inj)
        if it.size:
            pos, found = _lookup(c_code, cur[it])
            if not found.all():
                raise AssertionError("interpolated vertex is not a corner of a merged region")
            plo = c_par[pos]
            key = codec.decode(cur[it])
            for b in bits:
                w = np.ones(it.size)
                for a in range(d):
                    rel = key[:, a] - plo[:, a]          # 0, ps/2 or ps
                    up = np.where(rel == ps, 1.0, np.where(rel == 0, 0.0, 0.5))
                    w = w * (up if b[a] else 1.0 - up)
                rows.append(it)
                ccode.append(codec.encode(plo + b[None, :] * ps))
                vals.append(w)
        P, codes_next = _drop_zero_columns(np.concatenate(rows), np.concatenate(ccode),
                                           np.concatenate(vals), n_cur)
        prolong.append(P)
        level_codes.append(codes_next)
        regions.append((new_depth, new_lo))
        reg_depth, reg_lo = new_depth, new_lo

    return TreeLevels(m, M, capacity, Dmax, codec, level_codes, prolong, regions)
