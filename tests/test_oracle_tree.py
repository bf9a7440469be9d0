"""Pins of the oracle's keys, sort, tree, groups and neighbour sets (Sect. 3.1-3.2).

* keys: hand-worked values, and the octant path obtained by recursive
  bisection of the cube (a different computation from the oracle's
  quantise-and-interleave);
* sort: numpy's stable argsort;
* tree / groups: a set-based construction straight from the definition
  (a cell exists iff its parent holds more than the threshold), compared
  node by node, plus structural invariants;
* neighbour sets: brute force O(N^2) and scipy's periodic k-d tree.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from paper_1909_07439_amd import inputs

UNIT = dict(inputs.DEFAULTS, box_lo=(0.0, 0.0, 0.0), box_len=(1.0, 1.0, 1.0), periodic=(1, 1, 1))


def P(**kw):
    d = dict(UNIT)
    d.update(kw)
    return oracle.make_params(d)


def test_keys_hand_values():
    p = P()
    s = 2.0 ** -21
    x = np.array([0.0, s, 0.0, 0.0, 1.0 - 1e-12, 0.5, 0.25])
    y = np.array([0.0, 0.0, s, 0.0, 1.0 - 1e-12, 0.0, 0.0])
    z = np.array([0.0, 0.0, 0.0, s, 1.0 - 1e-12, 0.0, 0.0])
    k = oracle.keys(x, y, z, p)
    assert k[0] == 0
    assert k[1] == 4  # lowest x bit -> key bit 2
    assert k[2] == 2  # lowest y bit -> key bit 1
    assert k[3] == 1  # lowest z bit -> key bit 0
    assert k[4] == (1 << 63) - 1
    assert k[5] == 1 << 62  # top x bit -> key bit 62
    assert k[6] == 1 << 59


def test_keys_clamp_outside_box():
    p = P(periodic=(0, 0, 0))
    k = oracle.keys(np.array([-0.5, 1.5]), np.array([0.5, 0.5]), np.array([0.5, 0.5]), p)
    kin = oracle.keys(np.array([0.0, 1.0 - 1e-15]), np.array([0.5, 0.5]), np.array([0.5, 0.5]), p)
    assert k[0] == kin[0] and k[1] == kin[1]


def test_keys_follow_recursive_bisection():
    rng = np.random.default_rng(7)
    n = 300
    x, y, z = rng.random(n), rng.random(n), rng.random(n)
    k = oracle.keys(x, y, z, P())
    for i in range(n):
        lo = np.zeros(3)
        size = 1.0
        path = 0
        c = np.array([x[i], y[i], z[i]])
        for _ in range(21):
            size *= 0.5
            bits = (c >= lo + size).astype(np.uint64)
            lo = lo + size * bits
            path = (path << 3) | int(bits[0] << 2 | bits[1] << 1 | bits[2])
        assert path == int(k[i])


def test_keys_noncubic_box_uses_largest_side():
    p = P(box_lo=(-0.5, -1 / 32, -1 / 32), box_len=(1.0, 1 / 16, 1 / 16))
    k = oracle.keys(np.array([0.0]), np.array([1 / 32 - 1e-9]), np.array([-1 / 32]), p)
    # y sits just below lo+1/16 of a cube of side 1: y-index < 2^21/16
    iy = 0
    for b in range(21):
        iy |= ((int(k[0]) >> (3 * b + 1)) & 1) << b
    assert iy == int(np.floor((1 / 16 - 1e-9) * 2 ** 21))


def test_sort_is_stable_argsort():
    rng = np.random.default_rng(3)
    k = rng.integers(0, 50, 2000).astype(np.uint64)  # many ties
    np.testing.assert_array_equal(oracle.sort(k), np.argsort(k, kind="stable"))


def expected_tree(skeys, thr):
    """Set-based construction: cell (l, p) is a node iff l == 0, or its parent
    (l-1, p>>3) holds more than thr particles.  Sorted by (level, prefix)."""
    skeys = skeys.astype(np.uint64)
    nodes = []
    counts = {}
    for lev in range(22):
        pref = skeys >> np.uint64(63 - 3 * lev) if lev > 0 else np.zeros_like(skeys)
        u, first, cnt = np.unique(pref, return_index=True, return_counts=True)
        for pp, f, c in zip(u, first, cnt):
            counts[(lev, int(pp))] = (int(f), int(c))
    for (lev, pp), (f, c) in sorted(counts.items()):
        if lev == 0 or counts[(lev - 1, pp >> 3)][1] > thr:
            nodes.append((lev, pp, f, c))
    return nodes


def _skeys(n, seed, dup=0):
    rng = np.random.default_rng(seed)
    x, y, z = rng.random(n), rng.random(n), rng.random(n)
    if dup:
        x[:dup] = x[0]
        y[:dup] = y[0]
        z[:dup] = z[0]
    k = oracle.keys(x, y, z, P())
    return k[oracle.sort(k)]


@pytest.mark.parametrize("n,thr,seed,dup", [(1, 16, 1, 0), (10, 16, 2, 0), (2000, 16, 3, 0),
                                            (3000, 8, 4, 0), (1500, 1, 5, 0), (600, 4, 6, 40)])
def test_tree_matches_definition(n, thr, seed, dup):
    sk = _skeys(n, seed, dup)
    t = oracle.tree(sk, thr)
    exp = expected_tree(sk, thr)
    assert len(exp) == t["level"].size
    got = list(zip(t["level"].tolist(), t["prefix"].tolist(), t["first"].tolist(),
                   t["count"].tolist()))
    assert got == exp
    # children are contiguous and partition their parent
    for k in range(t["level"].size):
        leaf = t["child_first"][k] < 0
        if leaf:
            assert t["count"][k] <= thr or t["level"][k] == 21
            assert t["n_child"][k] == 0
        else:
            cf, nc = t["child_first"][k], t["n_child"][k]
            assert 1 <= nc <= 8
            ch = slice(cf, cf + nc)
            assert np.all(t["level"][ch] == t["level"][k] + 1)
            assert t["first"][cf] == t["first"][k]
            assert t["count"][ch].sum() == t["count"][k]
            assert np.all(t["prefix"][ch] >> np.uint64(3) == t["prefix"][k])


def expected_groups(skeys, thr):
    """Group cells: the nodes of the chopped tree with <= thr particles;
    consecutive group cells under one parent are packed greedily into groups
    of <= thr particles, a child with more particles ending a pack; level-21
    cells with more (identical keys) are cut into chunks of thr."""
    nodes = expected_tree(skeys, thr)
    if nodes[0][3] <= thr:
        return [(0, nodes[0][3])]
    children = {}
    for lev, pp, f, c in nodes:
        if lev > 0:
            children.setdefault((lev - 1, pp >> 3), []).append((f, c))
    out = []
    for lev, pp, f, c in nodes:
        if c > thr and lev == 21:
            out.extend((s, min(thr, f + c - s)) for s in range(f, f + c, thr))
        if c <= thr or lev == 21:
            continue
        pack = None
        for cf, cc in sorted(children[(lev, pp)]):
            if cc > thr:
                if pack:
                    out.append(tuple(pack))
                pack = None
            elif pack and pack[1] + cc <= thr:
                pack[1] += cc
            else:
                if pack:
                    out.append(tuple(pack))
                pack = [cf, cc]
        if pack:
            out.append(tuple(pack))
    return sorted(out)


@pytest.mark.parametrize("n,thr,seed,dup", [(1, 8, 1, 0), (7, 8, 2, 0), (2500, 8, 3, 0),
                                            (2500, 16, 4, 0), (900, 3, 5, 50)])
def test_groups_match_definition(n, thr, seed, dup):
    sk = _skeys(n, seed, dup)
    g = oracle.groups(sk, thr)
    got = list(zip(g["first"].tolist(), g["count"].tolist()))
    assert got == expected_groups(sk, thr)
    assert g["count"].sum() == n
    assert np.all(g["first"][1:] == g["first"][:-1] + g["count"][:-1])


@pytest.mark.parametrize("mode", [0, 1])
def test_neighbours_tree_equals_brute(mode):
    c = inputs.lattice(12, jitter=0.3)
    rng = np.random.default_rng(11)
    h = c["h"] * rng.uniform(0.7, 1.4, c["n"])
    p = oracle.make_params(c)
    ob, ib = oracle.neighbours(c["x"], c["y"], c["z"], h, p, mode=mode, brute=True)
    ot, it = oracle.neighbours(c["x"], c["y"], c["z"], h, p, mode=mode, brute=False)
    np.testing.assert_array_equal(ob, ot)
    np.testing.assert_array_equal(ib, it)


@pytest.mark.parametrize("mode", [0, 1])
def test_neighbours_bracketed_by_kdtree(mode):
    """scipy's periodic k-d tree with radii 2h(1-1e-9) and 2h(1+1e-9) must
    bracket the oracle's strict r < 2h sets."""
    c = inputs.lattice(14, jitter=0.25)
    rng = np.random.default_rng(12)
    h = c["h"] * rng.uniform(0.8, 1.25, c["n"])
    p = oracle.make_params(c)
    off, idx = oracle.neighbours(c["x"], c["y"], c["z"], h, p, mode=mode)
    pts = np.stack([c["x"], c["y"], c["z"]], 1)
    kd = cKDTree(pts, boxsize=1.0)
    for i in range(0, c["n"], 7):
        got = set(idx[off[i]:off[i + 1]].tolist())
        if mode == 0:
            lo = set(kd.query_ball_point(pts[i], 2 * h[i] * (1 - 1e-9)))
            hi = set(kd.query_ball_point(pts[i], 2 * h[i] * (1 + 1e-9)))
        else:
            cand = kd.query_ball_point(pts[i], 2 * h.max() * (1 + 1e-9))
            cand = np.array(cand)
            d = np.linalg.norm(((pts[cand] - pts[i] + 0.5) % 1.0) - 0.5, axis=1)
            hm = np.maximum(h[i], h[cand])
            lo = set(cand[(d < 2 * hm * (1 - 1e-9)) & (cand != i)].tolist())
            hi = set(cand[(d < 2 * hm * (1 + 1e-9)) & (cand != i)].tolist())
        assert lo <= got <= hi
