"""GPU parity of the sparse domain decomposition (Sec. 3.4, eq. moe) through the
C-ABI against the oracle on the same seeded inputs.

  * kept cells and the experts' subdomain trees: bit-exact;
  * blended decode: the decode tolerances of each form in value units (value
    scale 3): FP32 3e-5 (1 + |v|), BF16 6e-2.  A gate-weighted average is a
    convex combination of the experts' outputs, so it keeps the largest expert
    error; the gates themselves are products of multiples of 1/(4 halo) and
    add at most a few FP32 ulps.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import mlp, moe, tree as T

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def scene(gpu_lib):
    grid = workloads.two_spheres_sdf()
    tr = gpu_lib.Tree(grid.to(DEV), (0, 0, 0), gpu_lib.SDF, 3.0)
    ijk, vals = T.active_set_dense(grid.numpy(), (0, 0, 0), T.SDF, 3.0)
    return tr, T.build(ijk, vals)


GRIDS = [((0, 0, 0), 64, 8), ((-5, 3, 17), 40, 8), ((0, 0, 0), 16, 8), ((1000, -2000, 7), 256, 8),
         ((-3, -3, -3), 24, 1)]


@pytest.mark.parametrize("origin,size,halo", GRIDS)
def test_subdomain_cells_match_oracle(gpu_lib, scene, origin, size, halo):
    tr, ot = scene
    got = gpu_lib.subdomain_cells(tr, origin, size, halo)
    want = moe.kept_cells(ot["ijk"], origin, size)
    assert np.array_equal(got, want.astype(np.int32))


@pytest.mark.parametrize("origin,size,halo", GRIDS[:2])
def test_tree_subdomain_matches_oracle(gpu_lib, scene, origin, size, halo):
    tr, ot = scene
    cells = moe.kept_cells(ot["ijk"], origin, size).tolist() + [[50, 50, 50]]  # the last one is empty
    for c in cells:
        sub = tr.subdomain(origin, size, halo, c)
        ex = sub.export()
        q, v = moe.subdomain_voxels(ot["ijk"], ot["values"], c, origin, size, halo)
        assert sub.info().n_voxels == len(q)
        if len(q) == 0:
            continue
        so = T.build(q, v)
        assert np.array_equal(ex["leaf_origin"], so["leaf_origin"])
        assert np.array_equal(ex["leaf_mask"], so["leaf_mask"])
        assert np.array_equal(ex["leaf_off"].astype(np.int64), so["leaf_off"])
        assert np.array_equal(ex["values"], so["values"].astype(np.float32))


def _experts(gpu_lib, cells, origin, size, halo, shape, prec, net=0):
    """One random-parameter expert per cell (network `net`: 0 regressor, value
    scale 3; 1 level-0 classifier, logits) and the oracle's description of it."""
    W, H, m = shape
    K = 2 * m
    shapes = mlp.layer_shapes(K, W, H, 1)
    models, oracle_experts = [], []
    for k, c in enumerate(cells):
        lo, D = gpu_lib.subdomain_box(origin, size, halo, c)
        theta = workloads.init_params(K, W, H, 1, seed=100 + k)
        if net == 1:  # logits of order 1, not 1e-2, so that most mask bits are decisive
            theta[-(W + 1):] *= 20.0
        B = workloads.pe_matrix(6) if m == 18 else workloads.ffm_matrix(m, 10.0, seed=200 + k)
        mdl = gpu_lib.Model({net: (W, H, m, 1)}, precision=prec, domain_lo=lo, domain_size=D, value_scale=3.0)
        mdl.set_params(net, theta)
        mdl.set_encoding(net, B)
        models.append(mdl)
        oracle_experts.append(dict(cell=c, theta=theta.astype(np.float64), shapes=shapes, B=B.astype(np.float64),
                                   lo=lo, D=D, scale=3.0 if net == 0 else 1.0))
    return models, oracle_experts


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("shape", [(64, 3, 18), (128, 4, 64)], ids=["64x3_pe6", "128x4_ffm64"])
def test_decode_moe_matches_oracle(gpu_lib, scene, prec, shape):
    tr, ot = scene
    origin, size, halo = (0, 0, 0), 64, 8
    p = gpu_lib.FP32 if prec == "fp32" else gpu_lib.BF16
    cells = gpu_lib.subdomain_cells(tr, origin, size, halo)
    assert len(cells) == 8
    models, ex = _experts(gpu_lib, cells, origin, size, halo, shape, p)
    got = gpu_lib.decode_moe(models, cells, origin, size, halo, tr).cpu().numpy().astype(np.float64)
    want = moe.decode_moe(ot["ijk"], ex, origin, size, halo)
    n_exp = sum(moe.gate(ot["ijk"], c, origin, size, halo) > 0 for c in cells)
    assert (n_exp == 8).sum() > 1000  # the blend of eight experts is exercised
    err = np.abs(got - want)
    if p == gpu_lib.FP32:
        assert np.all(err <= 3e-5 * (1 + np.abs(want)))
    else:
        assert np.max(err) <= 6e-2


def test_decode_moe_offset_grid_and_ragged_counts(gpu_lib, scene):
    """A grid offset from the lattice, cell edge 40 (not a multiple of 8), so
    that cells hold ragged voxel counts and buckets start mid-tile."""
    tr, ot = scene
    origin, size, halo = (-5, 3, 17), 40, 8
    cells = gpu_lib.subdomain_cells(tr, origin, size, halo)
    models, ex = _experts(gpu_lib, cells, origin, size, halo, (64, 3, 18), gpu_lib.FP32)
    got = gpu_lib.decode_moe(models, cells, origin, size, halo, tr).cpu().numpy().astype(np.float64)
    want = moe.decode_moe(ot["ijk"], ex, origin, size, halo)
    assert np.all(np.abs(got - want) <= 3e-5 * (1 + np.abs(want)))


def test_decode_moe_many_pairs_per_voxel(gpu_lib, scene):
    """Cells of edge 16 with an 8-voxel halo: every voxel lies in the overlap of
    several widened boxes (more than two pairs per voxel on average), so the
    grouped decode's first pair buffers overflow, the routing writes nothing past
    them, and the decode runs again with buffers of the exact size; the result
    matches the oracle's blend.  A second call reuses the grown buffers."""
    tr, ot = scene
    origin, size, halo = (0, 0, 0), 16, 8
    cells = gpu_lib.subdomain_cells(tr, origin, size, halo)
    models, ex = _experts(gpu_lib, cells, origin, size, halo, (64, 3, 18), gpu_lib.FP32)
    n_exp = sum(moe.gate(ot["ijk"], c, origin, size, halo) > 0 for c in cells)
    assert n_exp.mean() > 2.5
    want = moe.decode_moe(ot["ijk"], ex, origin, size, halo)
    for _ in range(2):
        got = gpu_lib.decode_moe(models, cells, origin, size, halo, tr).cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - want) <= 3e-5 * (1 + np.abs(want)))


def test_decode_moe_single_expert_equals_decode(gpu_lib):
    """One cell whose gate is 1 on every voxel: the blend returns the expert's
    own decode exactly."""
    grid = workloads.sphere_sdf()
    tr = gpu_lib.Tree(grid.to(DEV), (0, 0, 0), gpu_lib.SDF, 3.0)
    origin, size, halo = (0, 0, 0), 64, 4
    cells = gpu_lib.subdomain_cells(tr, origin, size, halo)
    assert cells.tolist() == [[0, 0, 0]]
    for prec in (gpu_lib.FP32, gpu_lib.BF16):
        models, _ = _experts(gpu_lib, cells, origin, size, halo, (128, 4, 64), prec)
        got = gpu_lib.decode_moe(models, cells, origin, size, halo, tr).cpu().numpy()
        ref, _ = models[0].decode(tr, masks=False)
        assert np.array_equal(got.view(np.uint32), ref.cpu().numpy().view(np.uint32))


def test_moe_rejects_bad_arguments(gpu_lib, scene):
    tr, ot = scene
    origin = (0, 0, 0)
    cells = gpu_lib.subdomain_cells(tr, origin, 64, 8)
    models, _ = _experts(gpu_lib, cells, origin, 64, 8, (64, 3, 18), gpu_lib.FP32)
    for size, halo in [(64, 0), (15, 8)]:
        with pytest.raises(gpu_lib.NvdbError) as e:
            gpu_lib.subdomain_cells(tr, origin, size, halo)
        assert e.value.code == gpu_lib.E_INVALID
        with pytest.raises(gpu_lib.NvdbError) as e:
            gpu_lib.decode_moe(models, cells, origin, size, halo, tr)
        assert e.value.code == gpu_lib.E_INVALID
    # two experts for one cell
    dup = cells.copy()
    dup[1] = dup[0]
    with pytest.raises(gpu_lib.NvdbError) as e:
        gpu_lib.decode_moe(models, dup, origin, 64, 8, tr)
    assert e.value.code == gpu_lib.E_INVALID
    # voxels no expert covers (the second sphere's cell left out)
    keep = [k for k, c in enumerate(cells.tolist()) if c != [1, 0, 0]]
    with pytest.raises(gpu_lib.NvdbError) as e:
        gpu_lib.decode_moe([models[k] for k in keep], cells[keep], origin, 64, 8, tr)
    assert e.value.code == gpu_lib.E_INVALID
    # an expert without parameters
    bare = gpu_lib.Model({0: (64, 3, 18, 1)}, precision=gpu_lib.FP32, domain_size=80, value_scale=3.0)
    with pytest.raises(gpu_lib.NvdbError) as e:
        gpu_lib.decode_moe([bare] + models[1:], cells, origin, 64, 8, tr)
    assert e.value.code == gpu_lib.E_STATE
    # the library still works after the errors
    assert gpu_lib.decode_moe(models, cells, origin, 64, 8, tr).shape[0] == tr.info().n_voxels


def test_decode_moe_full_size_sampled(gpu_lib):
    """The benchmark's configuration: the 512^3 level set (2,994,515 voxels) in
    256^3 cells with an 8-voxel halo, eight BF16 4x128 experts (K 128), one
    blended decode of every voxel; 4096 sampled voxels checked against the
    oracle, half of them where two or more experts blend."""
    grid = workloads.noise_sphere_sdf(512, center=(256.0, 256.0, 256.0), radius=200.0, amplitude=20.0, octaves=4,
                                      scale=64.0, seed=0, device=DEV)
    ijk, vals = T.active_set_dense(grid.cpu().numpy(), (0, 0, 0), T.SDF, 3.0)
    ot = T.build(ijk, vals)
    tr = gpu_lib.Tree(grid, (0, 0, 0), T.SDF, 3.0)
    origin, size, halo = (0, 0, 0), 256, 8
    cells = gpu_lib.subdomain_cells(tr, origin, size, halo)
    assert np.array_equal(cells, moe.kept_cells(ot["ijk"], origin, size).astype(np.int32))
    models, ex = _experts(gpu_lib, cells, origin, size, halo, (128, 4, 64), gpu_lib.BF16)
    got = gpu_lib.decode_moe(models, cells, origin, size, halo, tr).cpu().numpy().astype(np.float64)
    n_exp = sum(moe.gate(ot["ijk"], c, origin, size, halo) > 0 for c in cells)
    rng = np.random.default_rng(7)
    multi = np.flatnonzero(n_exp >= 2)
    sel = np.concatenate([rng.choice(multi, 2048, replace=False),
                          rng.choice(len(ot["ijk"]), 2048, replace=False)])
    want = moe.decode_moe(ot["ijk"][sel], ex, origin, size, halo)
    assert np.max(np.abs(got[sel] - want)) <= 6e-2
    assert np.all(np.isfinite(got))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fit_experts_equals_sequential_fits(gpu_lib, scene, prec):
    """Experts fitted together (shared launches) end bit-identical to the same fits
    run one after the other, with the same losses (the kernels are
    deterministic and the fits share nothing)."""
    tr, _ = scene
    p = gpu_lib.FP32 if prec == "fp32" else gpu_lib.BF16
    origin, size, halo = (0, 0, 0), 64, 8
    cells = gpu_lib.subdomain_cells(tr, origin, size, halo)[:5]
    trees = [tr.subdomain(origin, size, halo, c) for c in cells]
    a, _ = _experts(gpu_lib, cells, origin, size, halo, (64, 3, 18), p)
    b, _ = _experts(gpu_lib, cells, origin, size, halo, (64, 3, 18), p)
    la = np.stack([m.fit(t, steps=30, batch=4096, nets_mask=1, seed=3) for m, t in zip(a, trees)])
    lb = gpu_lib.fit_experts(b, trees, steps=30, batch=4096, nets_mask=1, seed=3, return_losses=True)
    for ma, mb in zip(a, b):
        assert np.array_equal(ma.get_params(0).view(np.uint32), mb.get_params(0).view(np.uint32))
    assert np.array_equal(la[:, 0], lb[:, 0])
    assert np.all(np.isfinite(lb[:, 0])) and np.all(lb[:, 0, -5:].mean(1) < lb[:, 0, :3].mean(1))
    # a second round continues from the step counters, as nvdb_fit does
    for m, t in zip(a, trees):
        m.fit(t, steps=5, batch=4096, nets_mask=1, seed=3, return_losses=False)
    gpu_lib.fit_experts(b, trees, steps=5, batch=4096, nets_mask=1, seed=3)
    for ma, mb in zip(a, b):
        assert np.array_equal(ma.get_params(0).view(np.uint32), mb.get_params(0).view(np.uint32))
    with pytest.raises(gpu_lib.NvdbError) as e:
        gpu_lib.fit_experts([b[0], b[0]], trees[:2], steps=1, batch=4096, nets_mask=1)
    assert e.value.code == gpu_lib.E_INVALID


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_decode_moe_mask_matches_oracle(gpu_lib, scene, prec):
    """Blended level-0 masks: every voxel slot of every leaf, bit = blended logit
    > 0, against the oracle's blend at the slot centres (slots whose logit lies
    within the forward tolerance of 0 may go either way)."""
    tr, ot = scene
    origin, size, halo = (0, 0, 0), 64, 8
    p = gpu_lib.FP32 if prec == "fp32" else gpu_lib.BF16
    cells = gpu_lib.subdomain_cells(tr, origin, size, halo)
    models, ex = _experts(gpu_lib, cells, origin, size, halo, (64, 3, 18), p, net=1)
    mk = gpu_lib.decode_moe_mask(models, cells, origin, size, halo, tr).cpu().numpy().view(np.uint64)
    L = len(ot["leaf_origin"])
    slots = (ot["leaf_origin"][:, None, :].astype(np.int64) + T.n0_to_offset(np.arange(512))[None]).reshape(-1, 3)
    lg = moe.decode_moe(slots, ex, origin, size, halo).reshape(L, 512)
    bits = np.unpackbits(mk.view(np.uint8), bitorder="little").reshape(L, 512).astype(bool)
    near = np.abs(lg) <= (1e-4 if p == gpu_lib.FP32 else 2e-2)
    assert near.mean() < 0.1
    assert not np.any((bits != (lg > 0)) & ~near)
    # a grid whose cells can cut a leaf is refused
    with pytest.raises(gpu_lib.NvdbError) as e:
        gpu_lib.decode_moe_mask(models, cells, (4, 0, 0), size, halo, tr)
    assert e.value.code == gpu_lib.E_INVALID
    # experts without a level-0 classifier
    reg, _ = _experts(gpu_lib, cells, origin, size, halo, (64, 3, 18), p, net=0)
    with pytest.raises(gpu_lib.NvdbError) as e:
        gpu_lib.decode_moe_mask(reg, cells, origin, size, halo, tr)
    assert e.value.code == gpu_lib.E_INVALID


def test_moe_empty_and_single_voxel(gpu_lib):
    """Edge cases: a tree with no active voxel (no cells, empty subdomain, empty
    decode) and a single voxel at negative coordinates near a cell corner of an
    offset grid (its one expert, blended with itself)."""
    empty = gpu_lib.Tree(torch.full((9, 10, 11), 50.0, device=DEV), (0, 0, 0), gpu_lib.SDF, 3.0)
    origin, size, halo = (0, 0, 0), 16, 8
    assert gpu_lib.subdomain_cells(empty, origin, size, halo).shape == (0, 3)
    assert empty.subdomain(origin, size, halo, (0, 0, 0)).info().n_voxels == 0
    models, _ = _experts(gpu_lib, np.zeros((1, 3), np.int32), origin, size, halo, (64, 3, 18), gpu_lib.FP32)
    assert gpu_lib.decode_moe(models, [[0, 0, 0]], origin, size, halo, empty).numel() == 0

    grid = torch.where(torch.arange(5 * 6 * 7).reshape(5, 6, 7) == 101, 0.0, 9.0)
    one = gpu_lib.Tree(grid.to(DEV), (-1, -1, -1), gpu_lib.SDF, 1.0)
    ijk, vals = T.active_set_dense(grid.numpy(), (-1, -1, -1), T.SDF, 1.0)
    assert len(ijk) == 1
    origin, size, halo = (-9, 0, 3), 16, 8
    cells = gpu_lib.subdomain_cells(one, origin, size, halo)
    assert np.array_equal(cells, moe.kept_cells(ijk, origin, size).astype(np.int32))
    sub = one.subdomain(origin, size, halo, cells[0])
    assert sub.info().n_voxels == 1
    models, ex = _experts(gpu_lib, cells, origin, size, halo, (64, 3, 18), gpu_lib.FP32)
    got = gpu_lib.decode_moe(models, cells, origin, size, halo, one).cpu().numpy().astype(np.float64)
    want = moe.decode_moe(ijk, ex, origin, size, halo)
    assert np.all(np.abs(got - want) <= 3e-5 * (1 + np.abs(want)))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_decode_moe_l1_matches_oracle(gpu_lib, scene, prec):
    """Blended level-1 classes: every leaf slot of the level-1 node, the experts'
    three logits blended with the gates at the slot centres, argmax against the
    oracle's blend (slots whose two largest blended logits lie within the forward
    tolerance may go either way), in one grouped launch and, with one FP32 expert
    among BF16 ones, one launch per expert.  A halo that is not a multiple of 8 is
    refused."""
    tr, ot = scene
    origin, size, halo = (0, 0, 0), 64, 8
    p = gpu_lib.FP32 if prec == "fp32" else gpu_lib.BF16
    cells = gpu_lib.subdomain_cells(tr, origin, size, halo)
    assert len(cells) == 8
    W_, H_, m_ = 64, 4, 64
    shapes = mlp.layer_shapes(2 * m_, W_, H_, 3)
    models, ex = [], []
    for k, c in enumerate(cells):
        lo, D = gpu_lib.subdomain_box(origin, size, halo, c)
        theta = workloads.init_params(2 * m_, W_, H_, 3, seed=300 + k)
        theta[-(3 * W_ + 3):] *= 20.0  # logits of order 1
        B = workloads.ffm_matrix(m_, 3.0, seed=400 + k)
        mdl = gpu_lib.Model({2: (W_, H_, m_, 3)}, precision=p, domain_lo=lo, domain_size=D, value_scale=3.0)
        mdl.set_params(2, theta)
        mdl.set_encoding(2, B)
        models.append(mdl)
        ex.append(dict(cell=c, theta=theta.astype(np.float64), shapes=shapes, B=B.astype(np.float64), lo=lo, D=D,
                       scale=1.0))
    got = gpu_lib.decode_moe_l1(models, cells, origin, size, halo, tr).cpu().numpy().reshape(-1)
    n = 4096 * len(ot["l1_origin"])
    slots = ot["l1_origin"][np.arange(n) >> 12].astype(np.int64) + T.n1_to_offset(np.arange(n) & 4095)
    cls, lg = moe.decode_moe_l1(slots, ex, origin, size, halo)
    srt = np.sort(lg, axis=1)
    tie = (srt[:, -1] - srt[:, -2]) <= (1e-4 if p == gpu_lib.FP32 else 6e-2)
    assert tie.mean() < 0.1
    n_exp = sum(moe.gate_leaf_slot(slots, c, origin, size, halo) > 0 for c in cells)
    assert (n_exp == 8).sum() > 0  # slots blended from eight experts are exercised
    assert np.all((got == cls) | tie), int(((got != cls) & ~tie).sum())
    with pytest.raises(gpu_lib.NvdbError) as e:
        gpu_lib.decode_moe_l1(models, cells, origin, size, 4, tr)
    assert e.value.code == gpu_lib.E_INVALID
    if p == gpu_lib.BF16:  # an FP32 expert among BF16 experts: different kernels, one launch per expert
        other = gpu_lib.Model({2: (W_, H_, m_, 3)}, precision=gpu_lib.FP32, domain_lo=ex[0]["lo"],
                              domain_size=ex[0]["D"], value_scale=3.0)
        other.set_params(2, ex[0]["theta"].astype(np.float32))
        other.set_encoding(2, ex[0]["B"].astype(np.float32))
        mixed = gpu_lib.decode_moe_l1([other] + models[1:], cells, origin, size, halo, tr).cpu().numpy().reshape(-1)
        assert np.all((mixed == cls) | tie), int(((mixed != cls) & ~tie).sum())
