"""Pins of the sparse-domain-decomposition oracle (Sec. 3.4, eq. moe): tent
values in closed form, partition of unity, the eight-expert bound, kept cells
by brute force, subdomain sizes of a dense block, the blend of constant
experts (linear interpolation across the overlap), and the single-expert case
reducing to the plain decode, for voxel values, level-1 classes and active-tile
values."""
import itertools

import numpy as np
import pytest

import workloads
from oracle import fit as F, mlp, moe, tree as T


def const_expert(cell, c, origin, S, h, K=8, W=16, H=2):
    """An expert whose output is the constant c: every weight zero, head bias c."""
    shapes = mlp.layer_shapes(K, W, H, 1)
    theta = np.zeros(mlp.param_count(K, W, H, 1))
    theta[-1] = c
    lo, D = moe.widened_box(cell, origin, S, h)
    return dict(cell=cell, theta=theta, shapes=shapes, B=np.zeros((K // 2, 3)), lo=lo, D=D, scale=1.0)


def test_tent_values_closed_form():
    # S = 16, h = 4, cell 0 at origin 0: widened box [-4, 20).  Along x with y, z
    # in the core interior [4, 12) the gate is the 1-D tent: (i + 1/2) / 8 over
    # the first 8 voxels, 1 over [4, 12), symmetric at the top, 0 outside.
    S, h = 16, 4
    xs = np.arange(-6, 23)
    p = np.stack([xs, np.full_like(xs, 8), np.full_like(xs, 5)], 1)
    g = moe.gate(p, (0, 0, 0), (0, 0, 0), S, h)
    want = {x: 0.0 for x in xs}
    for i in range(8):
        want[-4 + i] = (i + 0.5) / 8
        want[19 - i] = (i + 0.5) / 8
    for x in range(4, 12):
        want[x] = 1.0
    assert np.array_equal(g, np.array([want[x] for x in xs]))
    # the 3-D gate is the product of the three tents
    q = np.array([[-4, -4, 19], [3, 12, 8]])
    assert np.array_equal(moe.gate(q, (0, 0, 0), (0, 0, 0), S, h), [(0.5 / 8) ** 3, (7.5 / 8) ** 2])


def test_partition_of_unity_and_expert_count():
    # all 27 cells around cell 0 kept: on the widened box of cell 0 the gates sum
    # to 1, and a voxel meets 2 cells on each axis where it lies within h of a
    # core face ((p - o) mod S < h or >= S - h), else 1: at most 8.
    S, h, o = 16, 4, np.array([3, -5, 7])
    cells = list(itertools.product((-1, 0, 1), repeat=3))
    ax = [np.arange(o[d] - h, o[d] + S + h) for d in range(3)]
    p = np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(-1, 3)
    gs = np.stack([moe.gate(p, c, o, S, h) for c in cells])
    assert np.array_equal(gs.sum(0), np.ones(len(p)))
    r = np.mod(p - o, S)
    near = (r < h) | (r >= S - h)
    assert np.array_equal((gs > 0).sum(0), np.prod(1 + near, axis=1))
    assert (gs > 0).sum(0).max() == 8
    # gate > 0 exactly on the widened box
    for c in cells:
        assert np.array_equal(moe.gate(p, c, o, S, h) > 0, moe.in_widened_box(p, c, o, S, h))


def test_kept_cells_brute_force():
    rng = np.random.default_rng(3)
    S, o = 12, np.array([-7, 2, 5])
    ijk = np.unique(rng.integers(-40, 40, size=(300, 3)), axis=0)
    got = moe.kept_cells(ijk, o, S)
    want = []
    for c in itertools.product(range(-5, 5), repeat=3):
        lo = o + np.array(c) * S
        if any(all(lo[d] <= v[d] < lo[d] + S for d in range(3)) for v in ijk.tolist()):
            want.append(c)
    assert got.tolist() == [list(c) for c in want]
    # the cores partition the voxels: each lies in the core of its own cell only
    for c in got:
        lo = o + c * S
        inside = np.all((ijk >= lo) & (ijk < lo + S), axis=1)
        assert np.array_equal(inside, np.all(moe.core_cell(ijk, o, S) == c, axis=1))


def test_subdomain_sizes_of_a_dense_block():
    # a dense (2S)^3 block aligned with the grid: each of its 8 cells sees its
    # core plus one halo side per axis, (S + h)^3 voxels
    S, h, o = 16, 4, np.array([-8, 5, 3])
    ax = [np.arange(o[d], o[d] + 2 * S) for d in range(3)]
    p = np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(-1, 3)
    v = np.arange(len(p), dtype=np.float64)
    cells = moe.kept_cells(p, o, S)
    assert len(cells) == 8
    for c in cells:
        q, w = moe.subdomain_voxels(p, v, c, o, S, h)
        assert len(q) == (S + h) ** 3
        assert np.array_equal(p[w.astype(np.int64)], q)


def test_blend_of_constant_experts():
    # two cells along x with constant experts 1 and 3: the blend is 1 on the
    # first core, 3 on the second, and the linear interpolation over the 2h
    # overlap [S - h, S + h); next to dropped cells (x < h, x >= 2S - h, every
    # y, z face) the single expert's value is kept exactly.
    S, h, o = 16, 4, (0, 0, 0)
    ex = [const_expert((0, 0, 0), 1.0, o, S, h), const_expert((1, 0, 0), 3.0, o, S, h)]
    xs = np.arange(0, 2 * S)
    for y, z in [(8, 8), (0, 15), (2, 13)]:
        p = np.stack([xs, np.full_like(xs, y), np.full_like(xs, z)], 1)
        got = moe.decode_moe(p, ex, o, S, h)
        w = np.clip((xs + 0.5 - (S - h)) / (2 * h), 0, 1)
        assert np.allclose(got, 1.0 * (1 - w) + 3.0 * w, rtol=0, atol=1e-15)
        assert np.array_equal(got[xs < S - h], np.ones((xs < S - h).sum()))
        assert np.array_equal(got[xs >= S + h], np.full((xs >= S + h).sum(), 3.0))
    # a voxel that no expert covers has no value
    assert np.isnan(moe.decode_moe(np.array([[-5, 8, 8]]), ex, o, S, h)[0])


def test_single_expert_is_the_plain_decode():
    v = workloads.sphere_sdf().numpy()
    ijk, vals = T.active_set_dense(v, (0, 0, 0), T.SDF, 3.0)
    tr = T.build(ijk, vals)
    S, h, o = 64, 8, (0, 0, 0)
    assert moe.kept_cells(tr["ijk"], o, S).tolist() == [[0, 0, 0]]
    K, W, H = 36, 64, 3
    shapes = mlp.layer_shapes(K, W, H, 1)
    theta = workloads.init_params(K, W, H, 1, seed=4).astype(np.float64)
    B = mlp.pe_matrix(6)
    lo, D = moe.widened_box((0, 0, 0), o, S, h)
    e = dict(cell=(0, 0, 0), theta=theta, shapes=shapes, B=B, lo=lo, D=D, scale=3.0)
    got = moe.decode_moe(tr["ijk"], [e], o, S, h)
    want = F.decode_values(theta, shapes, B, tr, lo, D, T.SDF, 3.0)
    assert np.allclose(got, want, rtol=0, atol=1e-12)


def test_two_spheres_layout():
    # the workload for the blended decode: 8 kept 64^3 cells, voxels with 1, 2,
    # 4 and 8 experts, gates summing to 1 on every voxel
    v = workloads.two_spheres_sdf().numpy()
    ijk, _ = T.active_set_dense(v, (0, 0, 0), T.SDF, 3.0)
    cells = moe.kept_cells(ijk, (0, 0, 0), 64)
    assert len(cells) == 8
    g = np.stack([moe.gate(ijk, c, (0, 0, 0), 64, 8) for c in cells])
    assert set(np.unique((g > 0).sum(0)).tolist()) == {1, 2, 4, 8}
    assert np.allclose(g.sum(0), 1.0, rtol=0, atol=1e-15)


def test_geometry_checks():
    with pytest.raises(ValueError):
        moe.check_geometry(15, 8)
    with pytest.raises(ValueError):
        moe.check_geometry(16, 0)
    moe.check_geometry(16, 8)


def const3_expert(cell, logits, origin, S, h, K=8, W=16, H=2):
    """A level-1 expert whose three logits are constant: weights zero, head biases."""
    shapes = mlp.layer_shapes(K, W, H, 3)
    theta = np.zeros(mlp.param_count(K, W, H, 3))
    theta[-3:] = logits
    lo, D = moe.widened_box(cell, origin, S, h)
    return dict(cell=cell, theta=theta, shapes=shapes, B=np.zeros((K // 2, 3)), lo=lo, D=D, scale=1.0)


def test_leaf_slot_gate_closed_form():
    # S = 32, h = 8, cell 0 at origin 0: widened box [-8, 40), edge 48.  Slots at
    # x origins -8, 0, ..., 32 have centres -4, 4, ..., 36 (t = 4, 12, ..., 44 from
    # the lower face): gates 4/16, 12/16, 1, 1, 12/16, 4/16 along x; slots whose
    # block leaves the box get 0; the 3-D gate is the product over the axes.
    S, h = 32, 8
    xs = np.arange(-16, 48, 8)
    o = np.stack([xs, np.full_like(xs, 8), np.full_like(xs, 16)], 1)
    g = moe.gate_leaf_slot(o, (0, 0, 0), (0, 0, 0), S, h)
    want = {-16: 0.0, -8: 0.25, 0: 0.75, 8: 1.0, 16: 1.0, 24: 0.75, 32: 0.25, 40: 0.0}
    assert np.array_equal(g, np.array([want[x] for x in xs]))
    assert moe.gate_leaf_slot(np.array([[-8, -8, 32]]), (0, 0, 0), (0, 0, 0), S, h)[0] == 0.25 ** 3
    # neighbours' gates sum to 1 on every slot of cell 0's widened box (all 27 cells kept)
    cells = list(itertools.product((-1, 0, 1), repeat=3))
    ax = np.arange(-8, 40, 8)
    o = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    gs = np.stack([moe.gate_leaf_slot(o, c, (0, 0, 0), S, h) for c in cells])
    assert np.array_equal(gs.sum(0), np.ones(len(o)))


def test_level1_blend_of_constant_experts():
    # two cells along x: expert 0 says class 0 (logits 1, 0, 0), expert 1 class 2
    # (logits 0, 0, 2).  Blended logits (1 - w, 0, 2 w) with w expert 1's share:
    # class 2 wherever 2 w > 1 - w, i.e. w > 1/3; slot centres in the overlap
    # [S - h, S + h) = [24, 40) are 28 and 36, with w = 0.25 and 0.75.
    S, h, org = 32, 8, (0, 0, 0)
    ex = [const3_expert((0, 0, 0), [1.0, 0.0, 0.0], org, S, h), const3_expert((1, 0, 0), [0.0, 0.0, 2.0], org, S, h)]
    xs = np.arange(0, 64, 8)
    o = np.stack([xs, np.full_like(xs, 8), np.full_like(xs, 8)], 1)
    cls, lg = moe.decode_moe_l1(o, ex, org, S, h)
    assert cls.tolist() == [0, 0, 0, 0, 2, 2, 2, 2]
    assert np.allclose(lg[3], [0.75, 0.0, 0.5]) and np.allclose(lg[4], [0.25, 0.0, 1.5])


def test_level1_single_expert_is_the_plain_decode():
    v = workloads.sphere_sdf().numpy()
    tr = T.build(*T.active_set_dense(v, (0, 0, 0), T.SDF, 3.0))
    S, h, o = 64, 8, (0, 0, 0)
    K, W, H = 36, 64, 3
    shapes = mlp.layer_shapes(K, W, H, 3)
    theta = workloads.init_params(K, W, H, 3, seed=5).astype(np.float64)
    B = mlp.pe_matrix(6)
    lo, D = moe.widened_box((0, 0, 0), o, S, h)
    e = dict(cell=(0, 0, 0), theta=theta, shapes=shapes, B=B, lo=lo, D=D, scale=1.0)
    slots = tr["l1_origin"][np.arange(4096 * len(tr["l1_origin"])) >> 12] + T.n1_to_offset(np.arange(4096 * len(tr["l1_origin"])) & 4095)
    cls, lg = moe.decode_moe_l1(slots, [e], o, S, h)
    want = F.decode_l1(theta, shapes, B, tr, lo, D)
    # the level-1 node spans [0, 128)^3; the cell's widened box [-8, 72)^3 holds the
    # slots with origins up to 64 (9^3 of them), where the blend is the expert itself
    inside = np.all(slots + 8 <= 72, axis=1)
    assert inside.sum() == 729 and np.all(np.isnan(lg[~inside]))
    assert np.allclose(lg[inside], want[inside], rtol=0, atol=1e-12)
    assert np.array_equal(cls[inside], F.l1_classes(want[inside]))


def test_tiles_single_expert_is_the_plain_tile_decode():
    # the pruned fog's active tiles all lie in the one cell's widened box [-8, 72)^3,
    # so the blend is the expert itself: the plain tile decode of Sec. 3.3.1
    v = workloads.saturated_fog().numpy()
    tr = T.prune_tiles(T.build(*T.active_set_dense(v, (0, 0, 0), T.FOG, 0.05)))
    assert len(tr["tile_value"]) >= 4
    S, h, o = 64, 8, (0, 0, 0)
    K, W, H = 36, 64, 3
    shapes = mlp.layer_shapes(K, W, H, 1)
    theta = workloads.init_params(K, W, H, 1, seed=9).astype(np.float64)
    B = mlp.pe_matrix(6)
    lo, D = moe.widened_box((0, 0, 0), o, S, h)
    e = dict(cell=(0, 0, 0), theta=theta, shapes=shapes, B=B, lo=lo, D=D, scale=1.0)
    got = moe.decode_moe_tiles(tr["tile_origin"], [e], o, S, h)
    want = F.decode_tiles(theta, shapes, B, tr, lo, D, T.FOG, 0.05)
    assert np.allclose(got, want, rtol=0, atol=1e-12)
    # a value scale multiplies the output; a tile outside every box gets NaN
    e2 = dict(e, scale=2.5)
    assert np.allclose(moe.decode_moe_tiles(tr["tile_origin"], [e2], o, S, h), 2.5 * want, rtol=0, atol=1e-12)
    assert np.isnan(moe.decode_moe_tiles([[80, 0, 0]], [e], o, S, h)).all()


def test_tiles_blend_of_constant_experts():
    # two cells along x with constant outputs 1 and 3 (value scales 1 and 2, so
    # 1 and 6 in value units): the blend interpolates linearly across the overlap
    # [24, 40), slot centres 28 and 36 with expert 1's share 0.25 and 0.75
    S, h, org = 32, 8, (0, 0, 0)
    e0 = const_expert((0, 0, 0), 1.0, org, S, h)
    e1 = dict(const_expert((1, 0, 0), 3.0, org, S, h), scale=2.0)
    xs = np.arange(0, 64, 8)
    o = np.stack([xs, np.full_like(xs, 8), np.full_like(xs, 8)], 1)
    got = moe.decode_moe_tiles(o, [e0, e1], org, S, h)
    assert np.allclose(got, [1, 1, 1, 2.25, 4.75, 6, 6, 6], rtol=0, atol=1e-12)
    # the same gates as the level-1 blend: tile value = sum g c / sum g
    g = np.stack([moe.gate_leaf_slot(o, e["cell"], org, S, h) for e in (e0, e1)])
    assert np.allclose(got, (g[0] * 1.0 + g[1] * 6.0) / g.sum(0), rtol=0, atol=1e-12)
