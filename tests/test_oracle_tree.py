"""Pins of the oracle's octree and lists (Sec. 2.1, Sec. 4 notation table,
Definition of HODLR3D admissibility, Algorithms 1 and 2).

- Morton codes: known values and round trips.
- Box relations: hand-picked V/E/F/W pairs (Sec. 3.1 figure of interactions).
- Depth rule and leaf contents: crafted clouds; every point lies geometrically
  inside its leaf; points of a leaf keep ascending original index.
- Partition: a pair-centric brute force (walk the levels for every pair of
  leaves and find where the two boxes first become V or W related) must give
  exactly the oracle's far blocks and near pairs; every ordered point pair is
  covered exactly once.
- Closed-form block counts for full trees, the paper's counts at L = 1 and the
  exact structure of the 16^3 grid with leaves of 64 points.
"""
import json
import os

import numpy as np
import pytest

from paper_2307_16303_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CUBE = dict(box_lo=inputs.CUBE_LO, box_side=inputs.CUBE_SIDE)


def test_morton_known_values(oracle_mod):
    assert oracle_mod.morton_encode((1, 0, 0), 1) == 4
    assert oracle_mod.morton_encode((0, 1, 0), 1) == 2
    assert oracle_mod.morton_encode((0, 0, 1), 1) == 1
    assert oracle_mod.morton_encode((3, 3, 3), 2) == 63
    assert oracle_mod.morton_encode((2, 0, 0), 2) == 32
    # (1,2,3) at 2 bits: high triple (0,1,1)=3, low triple (1,0,1)=5 -> 3*8+5
    assert oracle_mod.morton_encode((1, 2, 3), 2) == 29
    rng = np.random.default_rng(0)
    for _ in range(200):
        bits = int(rng.integers(1, 11))
        q = rng.integers(0, 2 ** bits, 3)
        assert oracle_mod.morton_decode(oracle_mod.morton_encode(q, bits), bits) == tuple(q)


def test_relations_hand_picked(oracle_mod):
    x = (2, 2, 2)
    assert oracle_mod.relation(x, x) == "self"
    assert oracle_mod.relation(x, (1, 2, 2)) == "F"
    assert oracle_mod.relation(x, (0, 2, 2)) == "W"  # one box away along an axis
    assert oracle_mod.relation(x, (3, 3, 2)) == "E"
    assert oracle_mod.relation(x, (3, 3, 3)) == "V"
    assert oracle_mod.relation(x, (1, 1, 1)) == "V"
    assert oracle_mod.relation(x, (4, 3, 3)) == "W"
    assert oracle_mod.relation(x, (2, 2, 5)) == "W"


def _leaf_geometry_ok(h, pts):
    lo, side = h.box()
    L = h.depth
    perm, leaf_off = h.tree()
    w = side / 2 ** L
    for b in range(8 ** L):
        idx = perm[leaf_off[b]:leaf_off[b + 1]]
        if idx.size == 0:
            continue
        q = np.array(inputs_morton_decode(b, L))
        p = pts[idx]
        assert np.all(p >= lo + q * w - 1e-12 * side)
        upper = lo + (q + 1) * w
        last = q == 2 ** L - 1
        assert np.all((p < upper) | last[None, :] & (p <= upper + 1e-12 * side))
        assert np.all(np.diff(idx) > 0)  # ascending original index inside a leaf
    assert sorted(perm.tolist()) == list(range(len(pts)))


def inputs_morton_decode(key, bits):
    # plain bit walk (independent of the oracle's decoder)
    x = y = z = 0
    for b in range(bits - 1, -1, -1):
        x = (x << 1) | ((key >> (3 * b + 2)) & 1)
        y = (y << 1) | ((key >> (3 * b + 1)) & 1)
        z = (z << 1) | ((key >> (3 * b)) & 1)
    return x, y, z


def test_depth_rule(oracle_mod):
    pts = inputs.uniform_points(10, seed=1)
    assert oracle_mod.HODLR3D(pts, leaf_size=10, compress=False, **CUBE).depth == 0
    assert oracle_mod.HODLR3D(pts, leaf_size=9, compress=False, **CUBE).depth >= 1
    # two points in opposite octants with one point per leaf -> L = 1
    two = np.array([[-0.5, -0.5, -0.5], [0.5, 0.5, 0.5]])
    h = oracle_mod.HODLR3D(two, leaf_size=1, compress=False, **CUBE)
    assert h.depth == 1 and h.num_far == 2 and h.num_near == 2
    # 16^3 grid, at most 64 per leaf -> L = 2 with exactly 64 points per leaf
    g = inputs.grid_points(16)
    h = oracle_mod.HODLR3D(g, leaf_size=64, compress=False, **CUBE)
    perm, leaf_off = h.tree()
    assert h.depth == 2
    np.testing.assert_array_equal(np.diff(leaf_off), 64)
    # with at most 63 per leaf it needs one more level (8 per leaf)
    h3 = oracle_mod.HODLR3D(g, leaf_size=63, compress=False, **CUBE)
    assert h3.depth == 3
    np.testing.assert_array_equal(np.diff(h3.tree()[1]), 8)
    # all points coincident: no depth separates them
    same = np.zeros((5, 3))
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.HODLR3D(same, leaf_size=2, max_depth=6, compress=False)


@pytest.mark.parametrize("n,leaf,seed", [(300, 4, 0), (1000, 16, 1), (64, 1, 2)])
def test_leaf_geometry(oracle_mod, n, leaf, seed):
    pts = inputs.uniform_points(n, seed=seed)
    h = oracle_mod.HODLR3D(pts, leaf_size=leaf, compress=False, **CUBE)
    _leaf_geometry_ok(h, pts)
    hb = oracle_mod.HODLR3D(pts, leaf_size=leaf, compress=False)  # smallest enclosing cube
    _leaf_geometry_ok(hb, pts)
    _, leaf_off = hb.tree()
    assert np.diff(leaf_off).max() <= leaf


def _rel(a, b):
    d = np.abs(np.array(a) - np.array(b))
    if d.max() == 0:
        return "self"
    if d.max() >= 2:
        return "W"
    return {3: "V", 2: "E", 1: "F"}[int(d.sum())]


def _brute_partition(h):
    """Pair-centric classification of every pair of non-empty leaves."""
    L = h.depth
    _, leaf_off = h.tree()
    cnt = np.diff(leaf_off)
    leaves = [b for b in range(8 ** L) if cnt[b] > 0]
    coords = {b: inputs_morton_decode(b, L) for b in leaves}
    far, near = set(), set()
    for a in leaves:
        for b in leaves:
            sep = None
            for l in range(1, L + 1):
                sh = L - l
                ca = tuple(c >> sh for c in coords[a])
                cb = tuple(c >> sh for c in coords[b])
                if _rel(ca, cb) in ("V", "W"):
                    sep = (l, a >> (3 * sh), b >> (3 * sh))
                    break
            if sep is None:
                near.add((a, b))
            else:
                far.add(sep)
    return far, near


@pytest.mark.parametrize("n,leaf,seed", [(400, 6, 3), (700, 5, 4), (150, 2, 5)])
def test_partition_matches_brute_force(oracle_mod, n, leaf, seed):
    pts = inputs.uniform_points(n, seed=seed)
    h = oracle_mod.HODLR3D(pts, leaf_size=leaf, compress=False, **CUBE)
    far_bf, near_bf = _brute_partition(h)
    f = h.far()
    far_or = set(zip(f["level"].tolist(), f["t"].tolist(), f["s"].tolist()))
    nr = h.near()
    near_or = set(zip(nr["t"].tolist(), nr["s"].tolist()))
    assert len(far_or) == h.num_far and len(near_or) == h.num_near
    assert far_or == far_bf
    assert near_or == near_bf
    # ordering: far by (level, t, s); near by (t, s)
    key = f["level"] * 8 ** 12 + f["t"] * 8 ** 6 + f["s"]
    assert np.all(np.diff(key) > 0)
    assert np.all(np.diff(nr["t"] * 8 ** 6 + nr["s"]) > 0)
    # relation labels of the near list
    L = h.depth
    for t, s, r in zip(nr["t"], nr["s"], nr["rel"]):
        assert oracle_mod.REL_NAMES[int(r)] == _rel(inputs_morton_decode(t, L), inputs_morton_decode(s, L))
    # every ordered point pair covered exactly once
    perm, leaf_off = h.tree()
    cover = np.zeros((n, n), dtype=np.int32)
    for l, t, s in far_or:
        sp = 8 ** (L - l)
        cover[leaf_off[t * sp]:leaf_off[(t + 1) * sp], leaf_off[s * sp]:leaf_off[(s + 1) * sp]] += 1
    for t, s in near_or:
        cover[leaf_off[t]:leaf_off[t + 1], leaf_off[s]:leaf_off[s + 1]] += 1
    assert cover.min() == 1 and cover.max() == 1
    assert int((f["m"] * f["n"]).sum()) + sum(
        int(leaf_off[t + 1] - leaf_off[t]) * int(leaf_off[s + 1] - leaf_off[s]) for t, s in near_or
    ) == n * n


def _D(n):
    return 19 * n ** 3 - 30 * n ** 2 + 12 * n


@pytest.mark.parametrize("L", [1, 2, 3, 4])
def test_closed_form_counts_full_tree(oracle_mod, L):
    # 2 points per axis per leaf: (2 * 2^L)^3 grid, 8 points in every leaf
    g = inputs.grid_points(2 * 2 ** L)
    h = oracle_mod.HODLR3D(g, leaf_size=8, compress=False, **CUBE)
    assert h.depth == L
    n = 2 ** L
    assert h.num_near == _D(n)
    f = h.far()
    lv = f["level"]
    m, nn = f["m"], f["n"]
    # V blocks in total 8 (n-1)^3; W per level 64 D(n_l/2) - D(n_l) - V_l
    rel = []
    for l, t, s in zip(lv, f["t"], f["s"]):
        rel.append(_rel(inputs_morton_decode(t, l), inputs_morton_decode(s, l)))
    rel = np.array(rel)
    assert int((rel == "V").sum()) == 8 * (n - 1) ** 3
    for l in range(1, L + 1):
        nl = 2 ** l
        v_l = 8 * (nl - 1) ** 3 - 8 * (nl // 2 - 1) ** 3
        w_l = 64 * _D(nl // 2) - _D(nl) - v_l if l >= 2 else 0
        assert int(((lv == l) & (rel == "V")).sum()) == v_l
        assert int(((lv == l) & (rel == "W")).sum()) == w_l
    assert np.all(m == 8 ** (L - lv + 1)) and np.all(nn == m)


def test_paper_counts_at_L1(oracle_mod):
    with open(os.path.join(GOLDEN, "paper_block_counts_L1.json")) as f:
        gold = json.load(f)
    g = inputs.grid_points(4)  # 64 points, 8 per octant
    h = oracle_mod.HODLR3D(g, leaf_size=8, compress=False, **CUBE)
    assert h.depth == 1
    fr = h.far()
    assert h.num_near == gold["dense"]
    rel = [_rel(inputs_morton_decode(t, 1), inputs_morton_decode(s, 1)) for t, s in zip(fr["t"], fr["s"])]
    assert rel.count("V") == gold["vertex_lowrank"]
    assert rel.count("W") == gold["well_separated_lowrank"]


def test_grid4096_exact_structure(oracle_mod):
    g = inputs.grid_points(16)
    h = oracle_mod.HODLR3D(g, leaf_size=64, compress=False, **CUBE)
    f = h.far()
    assert h.depth == 2 and h.num_near == 784
    lv = f["level"]
    assert int((lv == 1).sum()) == 8 and np.all(f["m"][lv == 1] == 512)
    assert int((lv == 2).sum()) == 208 + 2592 and np.all(f["m"][lv == 2] == 64)
    dense_entries = 784 * 64 * 64
    assert dense_entries == 3_211_264
    assert dense_entries + 8 * 512 * 512 + 2800 * 64 * 64 == 4096 ** 2


def test_smallest_enclosing_cube(oracle_mod):
    """Box rule for general inputs (Sec. 2.1 encloses the points in one cube B):
    lower corner = componentwise minimum, side = the largest extent over the
    three axes; the point on the upper face of that axis falls into the last
    box (half-open boxes, upper face clamped)."""
    pts = np.array([[-0.3, 0.10, -1.00],
                     [0.5, 0.20, -0.50],
                     [0.1, 0.15, -0.75],
                     [0.2, 0.12, -0.90],
                     [-0.1, 0.18, -0.60]])
    h = oracle_mod.HODLR3D(pts, leaf_size=1, tol=1e-8, compress=False)
    lo, side = h.box()
    np.testing.assert_array_equal(lo, [-0.3, 0.10, -1.00])
    assert side == 0.8  # x extent 0.5 - (-0.3) is the largest (y 0.1, z 0.5)
    # the cube is the smallest one: a point on the face x = lo + side exists, and
    # it is placed in the last box along x at every level
    perm, leaf_off = h.tree()
    L = h.depth
    assert L >= 1
    leaf_of = np.empty(len(pts), dtype=np.int64)
    for b in range(8 ** L):
        leaf_of[perm[leaf_off[b]:leaf_off[b + 1]]] = b
    qx, _, _ = oracle_mod.morton_decode(int(leaf_of[1]), L)
    assert qx == 2 ** L - 1
    # one coincident cloud: side 1 (nothing to enclose), lower corner at the point
    h1 = oracle_mod.HODLR3D(np.array([[0.25, -0.5, 2.0]] * 3), leaf_size=4, tol=1e-8,
                            compress=False)
    lo1, side1 = h1.box()
    np.testing.assert_array_equal(lo1, [0.25, -0.5, 2.0])
    assert side1 == 1.0
    # the largest extent along z
    pts_z = np.array([[0.0, 0.0, 0.0], [0.1, 0.2, 3.0], [0.05, -0.1, 1.0]])
    hz = oracle_mod.HODLR3D(pts_z, leaf_size=1, tol=1e-8, compress=False)
    loz, sidez = hz.box()
    np.testing.assert_array_equal(loz, [0.0, -0.1, 0.0])
    assert sidez == 3.0
