"""GPU parity of the active tiles and the tile value regressor (Sec. 3.3.1)
against the oracle: pruning bit for bit, training losses, tile decode, the tile
error report and the top-down decode with tiles.  Tolerances as in
test_gpu_parity (FP32 losses 1e-5 relative, BF16 2e-2; FP32 forward
1e-6 (1 + |y|), BF16 forward 2e-3 (1 + |y|); FP8 3e-2)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import fit as F, mlp, moe, tree as T

pytestmark = pytest.mark.gpu
DEV = "cuda"
THR = 0.05


def _fog(n):
    c = n / 2.0
    return workloads.saturated_fog(n=n, center=(c, c + 3.0, c - 2.0), radius=0.44 * n, scale=n / 4.0)


def _pair(gpu_lib, v, origin=(0, 0, 0)):
    tr = gpu_lib.Tree(v.to(DEV), origin, T.FOG, THR).prune_tiles()
    ot = T.prune_tiles(T.build(*T.active_set_dense(v.numpy(), origin, T.FOG, THR)))
    return tr, ot


def _assert_same(tr, ot):
    ex, i = tr.export(), tr.info()
    assert (i.n_voxels, i.n_leaves, i.n_l1, i.n_tiles) == (len(ot["values"]), len(ot["leaf_origin"]),
                                                           len(ot["l1_origin"]), len(ot["tile_value"]))
    assert np.array_equal(ex["leaf_origin"], ot["leaf_origin"])
    assert np.array_equal(ex["leaf_mask"], ot["leaf_mask"])
    assert np.array_equal(ex["leaf_off"].astype(np.int64), ot["leaf_off"])
    assert np.array_equal(ex["values"].astype(np.float64), ot["values"])
    assert np.array_equal(ex["l1_child"], ot["l1_child"])
    k, val, act = tr.export_tiles()
    assert np.array_equal(k.astype(np.int64), ot["tile_l1"] * 4096 + ot["tile_n1"])
    assert np.array_equal(val.astype(np.float64), ot["tile_value"])
    assert np.array_equal(act, ot["l1_active"])


@pytest.fixture(scope="module")
def fog(gpu_lib):
    return _pair(gpu_lib, _fog(128))


@pytest.fixture(scope="module")
def terraces(gpu_lib):
    """Fog rounded down to quarters: active tiles of three different values."""
    v = workloads.saturated_fog(n=128, center=(64.0, 67.0, 62.0), radius=56.3, scale=32.0, levels=4, gain=1.1,
                                amplitude=0.05)
    return _pair(gpu_lib, v)


def test_prune_tiles_matches_oracle(gpu_lib, fog):
    tr, ot = fog
    print("fog 128^3: %d voxels, %d leaves, %d tiles" % (len(ot["values"]), len(ot["leaf_origin"]),
                                                        len(ot["tile_value"])))
    assert len(ot["tile_value"]) >= 100
    _assert_same(tr, ot)


def test_prune_tiles_ragged_negative_origin(gpu_lib):
    """A ragged grid at a negative origin spanning several level-1 and level-2 nodes."""
    v = _fog(150)[:, 7:141, 3:].contiguous()
    tr, ot = _pair(gpu_lib, v, origin=(-4100, 60, -97))
    assert len(ot["tile_value"]) > 0 and len(ot["l2_origin"]) > 1
    _assert_same(tr, ot)


def test_prune_tiles_hand_and_edge_cases(gpu_lib):
    """The hand-counted case of the oracle pins (two tiles, one in a level-1 node
    left without leaves), a leaf of +0 and -0 values that stays a leaf, a tree
    without tiles, the empty tree, and a second pruning (refused)."""
    def block(o, value):
        off = np.stack(np.meshgrid(*[np.arange(8)] * 3, indexing="ij"), -1).reshape(-1, 3)
        return np.asarray(o) + off, np.full(512, value)
    parts = [block((0, 0, 0), 0.75), block((8, 0, 0), 0.75), block((16, 0, 0), 0.75), block((0, 128, 0), 1.0),
             block((0, 0, 256), 0.0)]
    parts[1][1][100] = 0.5
    parts[2] = (parts[2][0][1:], parts[2][1][1:])
    parts[4][1][7] = -0.0
    ijk = np.concatenate([p[0] for p in parts]).astype(np.int32)
    val = np.concatenate([p[1] for p in parts]).astype(np.float32)
    sdf_rule = (T.SDF, 10.0)   # every listed voxel is active (|v| <= 10)
    tr = gpu_lib.Tree.from_sparse(torch.from_numpy(ijk).to(DEV), torch.from_numpy(val).to(DEV), *sdf_rule)
    tp = tr.prune_tiles()
    ot = T.prune_tiles(T.build(ijk, val.astype(np.float64)))
    assert len(ot["tile_value"]) == 2
    _assert_same(tp, ot)
    with pytest.raises(gpu_lib.NvdbError):
        tp.prune_tiles()
    # a tree without constant full leaves: the same arrays, no tiles
    v = workloads.sphere_sdf(n=40, center=(20.0, 21.0, 19.0), radius=12.0)
    t0 = gpu_lib.Tree(v.to(DEV), (0, 0, 0), T.SDF, 2.0)
    p0 = t0.prune_tiles()
    assert p0.info().n_tiles == 0
    a, b = t0.export(), p0.export()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    # the empty tree
    e = gpu_lib.Tree(torch.full((9, 10, 11), 50.0, device=DEV), (0, 0, 0), T.SDF, 3.0).prune_tiles()
    i = e.info()
    assert (i.n_voxels, i.n_leaves, i.n_tiles) == (0, 0, 0)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_tile_regressor_fit_decode_errors(gpu_lib, terraces, prec):
    """Tile value regressor (3x64, positional encoding): i.i.d. SplitMix64 batches
    over the tiles (three tile values), losses of 6 steps against the oracle
    drawing the same indices; then the decode at every tile and the tile error
    report."""
    tr, ot = terraces
    assert len(np.unique(ot["tile_value"])) >= 3
    W, H, m, c = 64, 3, 18, 1
    shapes = mlp.layer_shapes(2 * m, W, H, c)
    B = workloads.pe_matrix(6)
    th0 = workloads.init_params(2 * m, W, H, c, seed=31)
    p = gpu_lib.FP32 if prec == "fp32" else gpu_lib.BF16
    model = gpu_lib.Model({3: (W, H, m, c)}, precision=p, domain_size=128, value_scale=1.0)
    model.set_params(3, th0)
    model.set_encoding(3, B)
    L = model.fit(tr, steps=6, batch=2048, nets_mask=8, seed=13)[3]
    _, _, _, lo = F.train(th0.astype(np.float64), shapes, B.astype(np.float64), ot, "tile", (0, 0, 0), 128, T.FOG,
                          THR, steps=6, batch=2048, seed=13)
    rel = np.abs(L - lo) / lo
    assert rel[0] <= (1e-6 if p == gpu_lib.FP32 else 2e-2), (L, lo)
    assert np.max(rel) <= (1e-5 if p == gpu_lib.FP32 else 2e-2), (L, lo)
    th = model.get_params(3).astype(np.float64)
    got = model.decode_tiles(tr).cpu().numpy()
    want = F.decode_tiles(th, shapes, B.astype(np.float64), ot, (0, 0, 0), 128, T.FOG, THR)
    tol = 1e-6 if p == gpu_lib.FP32 else 2e-3
    assert np.all(np.abs(got - want) <= tol * (1 + np.abs(want))), np.abs(got - want).max()
    rep = gpu_lib.errors_tiles(tr, model.decode_tiles(tr))
    orep = F.errors_tiles(ot, got.astype(np.float64))
    assert rep["n"] == orep["n"] == len(ot["tile_value"])
    assert abs(rep["max_abs"] - orep["max_abs"]) <= 1e-6 and abs(rep["rms"] - orep["rms"]) <= 1e-9 * max(1, orep["rms"])
    if p == gpu_lib.BF16:
        g8 = model.decode_tiles(tr, fp8=True).cpu().numpy()
        w8 = F.decode_tiles(th, shapes, B.astype(np.float64), ot, (0, 0, 0), 128, T.FOG, THR, fp8=True)
        assert np.abs(g8 - w8).max() <= 3e-2


def test_tile_regressor_errors(gpu_lib, fog):
    tr, _ = fog
    m = gpu_lib.Model({0: (64, 3, 18, 1)}, precision=gpu_lib.FP32, domain_size=128, value_scale=1.0)
    with pytest.raises(gpu_lib.NvdbError):
        m.decode_tiles(tr)                      # no tile regressor in the model
    m2 = gpu_lib.Model({3: (64, 3, 18, 1)}, precision=gpu_lib.FP32, domain_size=128, value_scale=1.0)
    with pytest.raises(gpu_lib.NvdbError):
        m2.decode_tiles(tr)                     # parameters not set
    m2.set_params(3, workloads.init_params(36, 64, 3, 1, seed=2))
    m2.set_encoding(3, workloads.pe_matrix(6))
    t0 = gpu_lib.Tree(_fog(64).to(DEV), (0, 0, 0), T.FOG, THR)   # not pruned: no tiles to train on
    with pytest.raises(gpu_lib.NvdbError):
        m2.fit(t0, steps=1, batch=64, nets_mask=8, seed=1)
    assert m2.decode_tiles(t0).numel() == 0


def test_decode_topology_with_tiles(gpu_lib, fog):
    """Top-down decode (Sec. 3.3.1): level-1 classes -> active tiles valued by the
    tile regressor, leaves -> level-0 classifier -> voxel values; FP32 against the
    oracle's decode with the same weights.  Tile slots may differ only where the
    level-1 logits are within rounding of a tie; values at the common tiles agree
    to FP32 forward accuracy."""
    tr, ot = fog
    nets = {2: (64, 4, 64, 3), 0: (64, 3, 18, 1), 1: (64, 3, 18, 1), 3: (64, 3, 18, 1)}
    m = gpu_lib.Model(nets, precision=gpu_lib.FP32, domain_size=128, value_scale=1.0)
    Bs = {2: workloads.ffm_matrix(64, 2.0, seed=4), 0: workloads.pe_matrix(6), 1: workloads.pe_matrix(6),
          3: workloads.pe_matrix(6)}
    for k, (W_, H_, m_, c_) in nets.items():
        m.set_params(k, workloads.init_params(2 * m_, W_, H_, c_, seed=50 + k))
        m.set_encoding(k, Bs[k])
    m.fit(tr, steps=200, batch=4096, nets_mask=15, seed=1, lr=3e-3)
    pred = m.decode_topology(tr)
    keys, vals, act = pred.export_tiles()

    def net(k):
        W_, H_, m_, c_ = nets[k]
        return (m.get_params(k).astype(np.float64), mlp.layer_shapes(2 * m_, W_, H_, c_), Bs[k].astype(np.float64))
    o = F.decode_topology(ot, (0, 0, 0), 128, T.FOG, THR, 1.0, net(2), net(0), net(1), tile=net(3))
    lg = F.decode_l1(*net(2), ot, (0, 0, 0), 128)
    srt = np.sort(lg, axis=1)
    tie = (srt[:, -1] - srt[:, -2]) <= 1e-4
    diff = np.setxor1d(keys.astype(np.int64), o["tile_key"])
    assert np.all(tie[diff]), len(diff)
    assert len(keys) > 0
    common, ig, io = np.intersect1d(keys.astype(np.int64), o["tile_key"], return_indices=True)
    d = np.abs(vals[ig] - o["tile_value"][io])
    assert d.max() <= 1e-5 * (1 + np.abs(o["tile_value"][io]).max()), d.max()
    # the active-tile bits of the result are its tiles
    assert int(T.popcount64(act).sum()) == len(keys)
    # the tile error of the decoded values against the truth at the correctly placed tiles
    truth = dict(zip((ot["tile_l1"] * 4096 + ot["tile_n1"]).tolist(), ot["tile_value"]))
    hit = [i for i, k in enumerate(keys.tolist()) if k in truth]
    err = np.abs(vals[hit] - np.array([truth[keys[i]] for i in hit]))
    print("tiles: %d predicted, %d true, %d placed right; max err %.3g rms %.3g"
          % (len(keys), len(truth), len(hit), err.max(), np.sqrt(np.mean(err ** 2))))


def test_archive_with_tiles(gpu_lib, fog):
    """An archive of a tree with active tiles stores the level-1 and leaf masks and
    the tile value regressor; its decode places every tile and leaf exactly and
    values the tiles with the stored (16-bit) regressor.  Voxel patches, which
    would rebuild the tree from voxels, are refused for such a tree."""
    tr, ot = fog
    nets = {0: (64, 3, 18, 1), 3: (64, 3, 18, 1)}
    m = gpu_lib.Model(nets, precision=gpu_lib.BF16, domain_size=128, value_scale=1.0)
    for k, (W_, H_, m_, c_) in nets.items():
        m.set_params(k, workloads.init_params(2 * m_, W_, H_, c_, seed=80 + k))
        m.set_encoding(k, workloads.pe_matrix(6))
    m.fit(tr, steps=50, batch=2048, nets_mask=9, seed=3)
    with pytest.raises(gpu_lib.NvdbError):
        gpu_lib.archive_write(m, tr, 9, gpu_lib.STORE_F16, explicit_l1=True, patches=True)
    buf = gpu_lib.archive_write(m, tr, 9, gpu_lib.STORE_F16, explicit_l1=True, explicit_l0=True)
    dt, info = gpu_lib.archive_decode(buf)
    assert info.nets_mask == 9
    de, ex = dt.export(), tr.export()
    for key in ("leaf_origin", "leaf_mask", "leaf_off", "l1_origin", "l1_child"):
        assert np.array_equal(de[key], ex[key]), key
    k_d, v_d, a_d = dt.export_tiles()
    k_t, _, a_t = tr.export_tiles()
    assert np.array_equal(k_d, k_t) and np.array_equal(a_d, a_t) and len(k_t) == len(ot["tile_value"])
    # the stored networks: both rounded to binary16, as the reader holds them
    r = gpu_lib.Model(nets, precision=gpu_lib.BF16, domain_size=128, value_scale=1.0)
    for k in nets:
        r.set_params16(k, gpu_lib.STORE_F16, m.get_params16(k, gpu_lib.STORE_F16))
        r.set_encoding(k, workloads.pe_matrix(6))
    assert np.array_equal(v_d, r.decode_tiles(tr).cpu().numpy())
    want, _ = r.decode(tr, values=True, masks=False)
    assert np.array_equal(de["values"], want.cpu().numpy())


@pytest.mark.parametrize("batch", [0, 1000])
def test_query_with_tiles(gpu_lib, fog, batch):
    """Random access through the tiles (Sec. 3.3.1, 3.5): voxel hits get the
    regressor at the query position, queries inside an active tile get the tile
    regressor's value (bit-equal to the library's tile decode), the rest the
    background; hit flags 1 / 2 / 0; FP32 against the oracle."""
    tr, ot = fog
    nets = {0: (64, 3, 18, 1), 3: (64, 3, 18, 1)}
    m = gpu_lib.Model(nets, precision=gpu_lib.FP32, domain_size=128, value_scale=1.0)
    th = {k: workloads.init_params(36, 64, 3, 1, seed=90 + k) for k in nets}
    B = workloads.pe_matrix(6)
    for k in nets:
        m.set_params(k, th[k])
        m.set_encoding(k, B)
    rng = np.random.default_rng(11)
    t_pick = rng.integers(0, len(ot["tile_value"]), 300)
    q = np.concatenate([ot["tile_origin"][t_pick] + rng.uniform(0.0, 8.0, (300, 3)),
                        ot["ijk"][rng.integers(0, len(ot["ijk"]), 300)] + rng.uniform(0.0, 1.0, (300, 3)),
                        rng.uniform(-20.0, 150.0, (3000, 3)), [[np.nan, 1, 1], [1e12, 0, 0]]]).astype(np.float32)
    v, h = m.query(tr, torch.from_numpy(q).to(DEV), background=-1.0, batch=batch, return_hits=True)
    v, h = v.cpu().numpy(), h.cpu().numpy()
    shapes = mlp.layer_shapes(36, 64, 3, 1)
    want, whits = F.query_values(th[0].astype(np.float64), shapes, B.astype(np.float64), ot, (0, 0, 0), 128, T.FOG,
                                 THR, q.astype(np.float64), background=-1.0,
                                 tile=(th[3].astype(np.float64), shapes, B.astype(np.float64)))
    tq = F.query_tiles(ot, q.astype(np.float64))
    assert np.array_equal(h == 1, whits) and np.array_equal(h == 2, tq >= 0)
    assert np.all(h[:300] == 2) and np.all(h[300:600] == 1)
    assert np.all(np.abs(v - want) <= 1e-6 * (1 + np.abs(want))), np.abs(v - want).max()
    dec = m.decode_tiles(tr).cpu().numpy()
    assert np.array_equal(v[h == 2], dec[tq[h == 2]])
    assert np.all(v[h == 0] == -1.0)
    # a model without the tile regressor treats the tiles as misses
    r = gpu_lib.Model({0: nets[0]}, precision=gpu_lib.FP32, domain_size=128, value_scale=1.0)
    r.set_params(0, th[0])
    r.set_encoding(0, B)
    v0, h0 = r.query(tr, torch.from_numpy(q).to(DEV), background=-1.0, batch=batch, return_hits=True)
    h0 = h0.cpu().numpy()
    assert np.array_equal(h0, np.where(h == 1, 1, 0)) and np.all(v0.cpu().numpy()[h == 2] == -1.0)


def _tile_voxels(ot):
    off = np.stack(np.meshgrid(*[np.arange(8)] * 3, indexing="ij"), -1).reshape(-1, 3)
    return (ot["tile_origin"][:, None, :] + off[None]).reshape(-1, 3)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_decode_moe_tiles_matches_oracle(gpu_lib, fog, prec):
    """Blended active-tile values under the sparse domain decomposition (Sec.
    3.3.1 tiles, Sec. 3.4 gates): the kept cells count the tiles' voxels, each
    expert's tile value regressor (own box, value scale 1.5) runs at the tiles in
    its widened box, blended with the gates at the tile centres, against the
    oracle's blend; a halo that is not a multiple of 8 and tiles that no expert
    holds are refused, and a tree without tiles decodes to nothing."""
    tr, ot = fog
    origin, size, halo = (0, 0, 0), 48, 8
    cells = gpu_lib.subdomain_cells(tr, origin, size, halo)
    want_cells = moe.kept_cells(np.concatenate([ot["ijk"], _tile_voxels(ot)]), origin, size)
    assert np.array_equal(cells, want_cells.astype(np.int32))
    # an offset grid of 10-voxel cells: tiles straddle up to eight cores, and cells
    # meeting only tile regions are kept
    tv = _tile_voxels(ot)
    off = gpu_lib.subdomain_cells(tr, (3, -5, 2), 10, 4)
    assert np.array_equal(off, moe.kept_cells(np.concatenate([ot["ijk"], tv]), (3, -5, 2), 10).astype(np.int32))
    assert len(off) > len(moe.kept_cells(ot["ijk"], (3, -5, 2), 10))
    W, H, m = 64, 3, 18
    shapes = mlp.layer_shapes(2 * m, W, H, 1)
    B = workloads.pe_matrix(6)
    p = gpu_lib.FP32 if prec == "fp32" else gpu_lib.BF16
    models, ex = [], []
    for k, c in enumerate(cells):
        lo, D = gpu_lib.subdomain_box(origin, size, halo, c)
        theta = workloads.init_params(2 * m, W, H, 1, seed=500 + k)
        mdl = gpu_lib.Model({3: (W, H, m, 1)}, precision=p, domain_lo=lo, domain_size=D, value_scale=1.5)
        mdl.set_params(3, theta)
        mdl.set_encoding(3, B)
        models.append(mdl)
        ex.append(dict(cell=c, theta=theta.astype(np.float64), shapes=shapes, B=B.astype(np.float64), lo=lo, D=D,
                       scale=1.5))
    got = gpu_lib.decode_moe_tiles(models, cells, origin, size, halo, tr).cpu().numpy().astype(np.float64)
    want = moe.decode_moe_tiles(ot["tile_origin"], ex, origin, size, halo)
    n_exp = sum(moe.gate_leaf_slot(ot["tile_origin"], c, origin, size, halo) > 0 for c in cells)
    assert np.all(n_exp >= 1) and (n_exp >= 2).sum() > 0  # tiles blended from several experts
    tol = 3e-5 if p == gpu_lib.FP32 else 3e-3
    assert np.all(np.abs(got - want) <= tol * (1 + np.abs(want))), np.abs(got - want).max()
    if p == gpu_lib.BF16:  # an FP32 expert among BF16 ones: one decode launch per expert
        m0 = gpu_lib.Model({3: (W, H, m, 1)}, precision=gpu_lib.FP32, domain_lo=ex[0]["lo"], domain_size=ex[0]["D"],
                           value_scale=1.5)
        m0.set_params(3, ex[0]["theta"].astype(np.float32))
        m0.set_encoding(3, B)
        mixed = gpu_lib.decode_moe_tiles([m0] + models[1:], cells, origin, size, halo, tr).cpu().numpy()
        assert np.all(np.abs(mixed - want) <= tol * (1 + np.abs(want))), np.abs(mixed - want).max()
    with pytest.raises(gpu_lib.NvdbError) as e:
        gpu_lib.decode_moe_tiles(models, cells, origin, size, 4, tr)
    assert e.value.code == gpu_lib.E_INVALID
    # without the centre cell's expert the tiles deep in its core have no expert
    keep = [i for i, c in enumerate(cells) if tuple(c) != (1, 1, 1)]
    assert len(keep) == len(cells) - 1
    with pytest.raises(gpu_lib.NvdbError) as e:
        gpu_lib.decode_moe_tiles([models[i] for i in keep], cells[keep], origin, size, halo, tr)
    assert e.value.code == gpu_lib.E_INVALID
    plain = gpu_lib.Tree(_fog(64).to(DEV), (0, 0, 0), T.FOG, THR)
    assert gpu_lib.decode_moe_tiles(models, cells, origin, size, halo, plain).numel() == 0


@pytest.mark.parametrize("grid", [((0, 0, 0), 48, 8), ((3, -5, 2), 40, 8)], ids=["aligned", "offset"])
def test_tree_subdomain_with_tiles(gpu_lib, fog, grid):
    """Expert training sets of a tree with active tiles (Sec. 3.4 over the tiles of
    Sec. 3.3.1): the voxels and tile voxels inside a cell's widened box, built and
    pruned, against the oracle's build of the same voxels and its pruning, for
    every kept cell; on the offset grid the boxes cut tiles, which come back as
    leaves of the voxels inside."""
    tr, ot = fog
    origin, size, halo = grid
    tv = _tile_voxels(ot)
    all_ijk = np.concatenate([ot["ijk"], tv])
    all_val = np.concatenate([ot["values"], np.repeat(ot["tile_value"], 512)])
    cells = gpu_lib.subdomain_cells(tr, origin, size, halo)
    n_tiles = n_cut = 0
    for c in cells:
        sel = moe.in_widened_box(all_ijk, c, origin, size, halo)
        want = T.prune_tiles(T.build(all_ijk[sel], all_val[sel]))
        sub = tr.subdomain(origin, size, halo, c)
        _assert_same(sub, want)
        n_tiles += len(want["tile_value"])
        tin = moe.in_widened_box(tv, c, origin, size, halo).reshape(-1, 512).sum(1)
        n_cut += int(((tin > 0) & (tin < 512)).sum())
    assert n_tiles > len(ot["tile_value"])  # tiles in the overlaps belong to several experts
    if origin != (0, 0, 0):
        assert n_cut > 0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fit_tile_experts_equals_sequential_fits(gpu_lib, fog, prec):
    """Tile value regressors of the experts of a tree with active tiles (Sec. 3.3.1
    under Sec. 3.4), fitted together in shared launches, end bit-identical to the
    same fits run one after the other, with the same losses; then their blended
    decode equals the oracle's blend of the fitted parameters."""
    tr, ot = fog
    origin, size, halo = (0, 0, 0), 64, 8
    cells = gpu_lib.subdomain_cells(tr, origin, size, halo)
    subs = [tr.subdomain(origin, size, halo, c) for c in cells]
    keep = [i for i, s_ in enumerate(subs) if s_.info().n_tiles > 0]
    assert len(keep) == len(cells) == 8
    p = gpu_lib.FP32 if prec == "fp32" else gpu_lib.BF16
    W, H, m = 64, 3, 18
    B = workloads.pe_matrix(6)

    def experts():
        out = []
        for k, c in enumerate(cells):
            lo, D = gpu_lib.subdomain_box(origin, size, halo, c)
            md = gpu_lib.Model({3: (W, H, m, 1)}, precision=p, domain_lo=lo, domain_size=D, value_scale=1.0)
            md.set_params(3, workloads.init_params(2 * m, W, H, 1, seed=700 + k))
            md.set_encoding(3, B)
            out.append(md)
        return out
    a, b = experts(), experts()
    la = np.stack([md.fit(t, steps=20, batch=2048, nets_mask=8, seed=5)[3] for md, t in zip(a, subs)])
    lb = gpu_lib.fit_experts(b, subs, steps=20, batch=2048, nets_mask=8, seed=5, return_losses=True)[:, 3]
    for ma, mb in zip(a, b):
        assert np.array_equal(ma.get_params(3).view(np.uint32), mb.get_params(3).view(np.uint32))
    assert np.array_equal(la, lb) and np.all(np.isfinite(lb))
    shapes = mlp.layer_shapes(2 * m, W, H, 1)
    ex = []
    for c, md in zip(cells, b):
        lo, D = gpu_lib.subdomain_box(origin, size, halo, c)
        ex.append(dict(cell=c, theta=md.get_params(3).astype(np.float64), shapes=shapes, B=B.astype(np.float64),
                       lo=lo, D=D, scale=1.0))
    got = gpu_lib.decode_moe_tiles(b, cells, origin, size, halo, tr).cpu().numpy().astype(np.float64)
    want = moe.decode_moe_tiles(ot["tile_origin"], ex, origin, size, halo)
    tol = 3e-5 if p == gpu_lib.FP32 else 3e-3
    assert np.all(np.abs(got - want) <= tol * (1 + np.abs(want))), np.abs(got - want).max()
