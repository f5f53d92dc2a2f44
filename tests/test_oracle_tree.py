"""Pins of the oracle tree build (Sec. 3.1 VDB, Tab. memory_cost) against
brute force, invariants and the paper's printed byte accounting."""
import json
import math
import os

import numpy as np
import pytest

from oracle import tree as T

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_figures.json")))


def brute_build(ijk):
    """Dictionary-based reference using Python floor division (an independent route)."""
    leaves = {}
    for p in map(tuple, ijk):
        lo = tuple((c // 8) * 8 for c in p)
        n0 = ((p[0] - lo[0]) << 6) | ((p[1] - lo[1]) << 3) | (p[2] - lo[2])
        leaves.setdefault(lo, set()).add(n0)

    def key(lo):
        l2 = tuple((c // 4096) * 4096 for c in lo)
        n2 = (((lo[0] - l2[0]) // 128) << 10) | (((lo[1] - l2[1]) // 128) << 5) | ((lo[2] - l2[2]) // 128)
        l1 = tuple((c // 128) * 128 for c in lo)
        n1 = (((lo[0] - l1[0]) // 8) << 8) | (((lo[1] - l1[1]) // 8) << 4) | ((lo[2] - l1[2]) // 8)
        return l2 + (n2, n1)

    order = sorted(leaves, key=key)
    return order, leaves


def random_sparse(rng, n, spread):
    pts = set()
    centres = [rng.integers(-spread, spread, 3) for _ in range(4)]
    while len(pts) < n:
        c = centres[rng.integers(0, 4)]
        pts.add(tuple(int(v) for v in c + rng.integers(-20, 20, 3)))
    ijk = np.array(sorted(pts), dtype=np.int32)
    rng.shuffle(ijk)
    return ijk


@pytest.mark.parametrize("seed,spread", [(0, 50), (1, 5000), (2, 9000)])
def test_tree_matches_brute_force(seed, spread):
    rng = np.random.default_rng(seed)
    ijk = random_sparse(rng, 3000, spread)
    vals = rng.standard_normal(len(ijk))
    tr = T.build(ijk, vals)
    order, leaves = brute_build(ijk)
    assert [tuple(o) for o in tr["leaf_origin"]] == order
    for li, lo in enumerate(order):
        n0s = sorted(leaves[lo])
        a, b = tr["leaf_off"][li], tr["leaf_off"][li + 1]
        assert b - a == len(n0s)
        got = tr["ijk"][a:b] - np.array(lo)
        assert [((x << 6) | (y << 3) | z) for x, y, z in got] == n0s
        bits = [n for n in range(512) if (int(tr["leaf_mask"][li, n >> 6]) >> (n & 63)) & 1]
        assert bits == n0s
    # values travel with their coordinates
    lookup = {tuple(p): v for p, v in zip(ijk, vals)}
    assert np.array_equal(tr["values"], np.array([lookup[tuple(p)] for p in tr["ijk"]]))


def test_tree_invariants():
    rng = np.random.default_rng(5)
    ijk = random_sparse(rng, 5000, 6000)
    tr = T.build(ijk, np.zeros(len(ijk)))
    N, L = len(ijk), len(tr["leaf_origin"])
    assert int(T.popcount64(tr["leaf_mask"]).sum()) == N
    assert np.all(tr["leaf_origin"] % 8 == 0)
    assert np.all(tr["l1_origin"] % 128 == 0)
    assert np.all(tr["l2_origin"] % 4096 == 0)
    assert np.all(np.diff(tr["leaf_off"]) > 0) and tr["leaf_off"][-1] == N
    # (leaf, n0) <-> p is a bijection
    p = tr["leaf_origin"][tr["vox_leaf"]].astype(np.int64) + T.n0_to_offset(tr["vox_n0"])
    assert np.array_equal(p, tr["ijk"].astype(np.int64))
    assert len({tuple(q) for q in p}) == N
    # L1 child bits are exactly the existing leaves
    assert int(T.popcount64(tr["l1_child"]).sum()) == L
    for li in range(L):
        node = tr["leaf_l1"][li]
        o = tr["leaf_origin"][li] - tr["l1_origin"][node]
        n1 = ((o[0] // 8) << 8) | ((o[1] // 8) << 4) | (o[2] // 8)
        assert T.mask_bits(tr["l1_child"], [node], [n1])[0] == 1
    assert int(T.popcount64(tr["l2_child"]).sum()) == len(tr["l1_origin"])


def test_negative_coordinates_floor():
    d = T.decompose(np.array([[-1, -8, -9], [4095, 4096, -4097]], dtype=np.int32))
    assert d["leaf_origin"].tolist() == [[-8, -8, -16], [4088, 4096, -4104]]
    assert d["l1_origin"].tolist() == [[-128, -128, -128], [3968, 4096, -4224]]
    assert d["l2_origin"].tolist() == [[-4096, -4096, -4096], [0, 4096, -8192]]
    assert d["n0"].tolist() == [(7 << 6) | (0 << 3) | 7, (7 << 6) | (0 << 3) | 7]


def test_duplicates_rejected():
    with pytest.raises(ValueError):
        T.build(np.array([[1, 2, 3], [1, 2, 3]]), np.zeros(2))


def test_sphere_active_count_two_ways():
    """phi = |p - (32,32,32)| - 24 on [0,63]^3 with |phi| <= 3: 43,878 voxels."""
    count = 0
    for x in range(64):
        for y in range(64):
            for z in range(64):
                r = math.sqrt((x - 32) ** 2 + (y - 32) ** 2 + (z - 32) ** 2)
                count += abs(r - 24.0) <= 3.0
    # second route: integer squared radii, 21^2 <= r^2 <= 27^2
    g = np.indices((64, 64, 64)) - 32
    r2 = (g ** 2).sum(0)
    assert count == int(((r2 >= 21 ** 2) & (r2 <= 27 ** 2)).sum()) == 43878
    shell = 4.0 / 3.0 * math.pi * (27 ** 3 - 21 ** 3)
    assert abs(count - shell) / shell < 0.01


def test_sphere_tree_shape():
    import workloads
    v = workloads.sphere_sdf().numpy()
    ijk, vals = T.active_set_dense(v, (0, 0, 0), T.SDF, 3.0)
    tr = T.build(ijk, vals)
    assert len(vals) == 43878
    assert len(tr["leaf_origin"]) == 257 and len(tr["l1_origin"]) == 1 and len(tr["l2_origin"]) == 1


def test_byte_accounting_matches_paper():
    g = GOLDEN["memory_cost"]
    b = T.explicit_bytes(g["leaf_nodes"], g["l1_nodes"], g["l2_nodes"])
    assert b["l2"] == g["l2_bytes"]
    assert b["l1"] == g["l1_bytes"]
    assert b["leaf_mask"] == g["leaf_mask_bytes"]
    assert g["leaf_nodes"] * T.VOXELS_PER_LEAF == g["voxels"]
    assert b["voxels"] == g["voxel_bytes"]
    assert sum(b.values()) == g["total_bytes"]
    # [Hash,5,4,NN(3)]: voxels replaced by 4-byte parameters
    nn3 = b["l2"] + b["l1"] + b["leaf_mask"] + 4 * g["nn3_voxel_params"]
    assert 4 * g["nn3_voxel_params"] == g["nn3_voxel_bytes"] and nn3 == g["nn3_total_bytes"]
    assert round(100.0 * nn3 / g["total_bytes"], 3) == g["nn3_percent"]
    # [Hash,5,NN(4),NN(3)]: level-0 masks become parameters plus 12-byte coordinate patches
    assert 4 * g["nn4_l0_params"] + 12 * g["nn4_l0_patches"] == g["nn4_l0_bytes"]
    assert 4 * g["nn4_voxel_params"] == g["nn4_voxel_bytes"]
    total = g["l2_bytes"] + g["nn4_l1_bytes"] + g["nn4_l0_bytes"] + g["nn4_voxel_bytes"]
    assert total == g["nn4_total_bytes"]
    assert round(100.0 * total / g["total_bytes"], 3) == g["nn4_percent"]
    # the same column per level from the oracle's accounting, level-1 row included
    nb = T.neural_bytes(g["l2_nodes"], g["l1_nodes"], g["nn4_l1_params"], g["nn4_l1_patches"], g["nn4_l0_params"],
                        g["nn4_l0_patches"], g["nn4_voxel_params"])
    assert (nb["l2"], nb["l1"], nb["leaf_mask"], nb["voxels"]) == (g["l2_bytes"], g["nn4_l1_bytes"],
                                                                     g["nn4_l0_bytes"], g["nn4_voxel_bytes"])
    assert sum(nb.values()) == g["nn4_total_bytes"]


def test_active_set_sparse_rule_and_order():
    """Closed interval for level sets, strict threshold for fog; rows kept in input
    order; on a dense grid listed voxel by voxel it selects what the dense rule
    selects (brute force over a random grid)."""
    ijk = np.array([[0, 0, 0], [1, 2, 3], [-5, 7, 9], [4, 4, 4]], np.int32)
    v = np.array([3.0, -3.0, 3.0001, 0.5], np.float32)
    a, va = T.active_set_sparse(ijk, v, T.SDF, 3.0)
    assert a.tolist() == [[0, 0, 0], [1, 2, 3], [4, 4, 4]] and va.tolist() == [3.0, -3.0, 0.5]
    b, vb = T.active_set_sparse(ijk, v, T.FOG, 3.0)
    assert b.tolist() == [[-5, 7, 9]]
    rng = np.random.default_rng(4)
    grid = rng.normal(0, 2, (6, 5, 7)).astype(np.float32)
    org = (-3, 10, 4)
    for kind, thr in ((T.SDF, 1.0), (T.FOG, 0.7)):
        ref = set(map(tuple, T.active_set_dense(grid, org, kind, thr)[0].tolist()))
        pts = np.array([[i + org[0], j + org[1], k + org[2]] for i in range(6) for j in range(5) for k in range(7)])
        got, _ = T.active_set_sparse(pts, grid.reshape(-1), kind, thr)
        assert set(map(tuple, got.tolist())) == ref


# ---------------------------------------------------------------- active tiles (Sec. 3.3.1)
def _block(origin, value=0.75):
    o = np.asarray(origin, np.int64)
    off = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"), -1).reshape(-1, 3)
    return o + off, np.full(512, value, np.float64)


def _tile_case():
    """Four leaf-sized blocks: A (0,0,0) full and constant; B (8,0,0) full with one
    voxel of another value; C (16,0,0) constant with one voxel missing; D (0,128,0),
    in a second level-1 node, full and constant."""
    a, va = _block((0, 0, 0), 0.75)
    b, vb = _block((8, 0, 0), 0.75)
    vb[100] = 0.5
    c, vc = _block((16, 0, 0), 0.75)
    c, vc = c[1:], vc[1:]
    d, vd = _block((0, 128, 0), 1.0)
    return np.concatenate([a, b, c, d]).astype(np.int32), np.concatenate([va, vb, vc, vd])


def test_prune_tiles_hand_case():
    ijk, v = _tile_case()
    tr = T.prune_tiles(T.build(ijk, v))
    # two tiles (A, D) in canonical order, two leaves (B, C) left
    assert tr["tile_origin"].tolist() == [[0, 0, 0], [0, 128, 0]]
    assert tr["tile_value"].tolist() == [0.75, 1.0]
    assert tr["tile_n1"].tolist() == [0, 0]
    assert tr["tile_l1"].tolist() == [0, 1]
    assert tr["leaf_origin"].tolist() == [[8, 0, 0], [16, 0, 0]]
    assert len(tr["values"]) == 512 + 511 and tr["leaf_off"].tolist() == [0, 512, 1023]
    assert tr["vox_leaf"].tolist() == [0] * 512 + [1] * 511
    # level-1 node 0 (origin 0): children at n1 = 1 << 8 (x = 8) and 2 << 8 (x = 16), tile at n1 = 0;
    # node 1 (origin (0,128,0)): no child, a tile at n1 = 0
    assert tr["l1_origin"].tolist() == [[0, 0, 0], [0, 128, 0]]
    child = {(int(n), int(b)) for n in range(2) for b in range(4096) if T.mask_bits(tr["l1_child"], n, b)}
    active = {(int(n), int(b)) for n in range(2) for b in range(4096) if T.mask_bits(tr["l1_active"], n, b)}
    assert child == {(0, 256), (0, 512)}
    assert active == {(0, 0), (1, 0)}
    # +0 and -0 are different values: such a leaf stays a leaf
    e, ve = _block((0, 0, 256), 0.0)
    ve[7] = -0.0
    te = T.prune_tiles(T.build(e.astype(np.int32), ve))
    assert len(te["tile_value"]) == 0 and len(te["leaf_origin"]) == 1
    te = T.prune_tiles(T.build(e.astype(np.int32), np.zeros(512)))
    assert len(te["tile_value"]) == 1 and len(te["leaf_origin"]) == 0 and len(te["values"]) == 0
    # a tree without constant full leaves is unchanged
    tr0 = T.build(ijk[512:512 + 1023], v[512:512 + 1023])
    tp = T.prune_tiles(tr0)
    assert len(tp["tile_value"]) == 0 and np.array_equal(tp["values"], tr0["values"])
    assert np.array_equal(tp["l1_child"], tr0["l1_child"])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_prune_tiles_is_lossless(seed):
    """Expanding every tile back into its 512 voxels gives the original active set
    and values exactly, and no kept leaf is full and constant."""
    rng = np.random.default_rng(seed)
    ijk = random_sparse(rng, 3000, 60)
    vals = rng.choice([0.25, 0.5], size=len(ijk))
    blocks = [_block(tuple(int(c) for c in 8 * rng.integers(-8, 8, 3)), float(rng.choice([0.25, 1.0])))
              for _ in range(6)]
    pts = {tuple(p): float(x) for p, x in zip(ijk.tolist(), vals)}
    for bi, bv in blocks:
        for p, x in zip(bi.tolist(), bv):
            pts[tuple(p)] = x
    keys = sorted(pts)
    ijk = np.array(keys, np.int32)
    v = np.array([pts[k] for k in keys])
    tr = T.prune_tiles(T.build(ijk, v))
    assert len(tr["tile_value"]) >= 1
    back = {tuple(p): float(x) for p, x in zip(tr["ijk"].tolist(), tr["values"])}
    for o, x in zip(tr["tile_origin"], tr["tile_value"]):
        bi, bv = _block(o, x)
        for p in bi.tolist():
            assert tuple(p) not in back
            back[tuple(p)] = x
    assert back == pts
    for i in range(len(tr["leaf_origin"])):
        seg = tr["values"][tr["leaf_off"][i]:tr["leaf_off"][i + 1]]
        assert not (len(seg) == 512 and np.all(seg == seg[0]))
    # every tile sits at an active-tile bit, no child bit there
    for n, b in zip(tr["tile_l1"], tr["tile_n1"]):
        assert T.mask_bits(tr["l1_active"], n, b) == 1 and T.mask_bits(tr["l1_child"], n, b) == 0
    assert int(T.popcount64(tr["l1_active"]).sum()) == len(tr["tile_value"])
