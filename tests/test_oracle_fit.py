"""Pins of the oracle fit/decode/error path: sample construction, an Adam
fit that lowers the loss, and the error report on known cases."""
import numpy as np
import pytest

import workloads
from oracle import fit as F, mlp, tree as T


@pytest.fixture(scope="module")
def sphere():
    v = workloads.sphere_sdf().numpy()
    ijk, vals = T.active_set_dense(v, (0, 0, 0), T.SDF, 3.0)
    return T.build(ijk, vals)


def test_net_inputs(sphere):
    tr = sphere
    # regressor: voxel centres and scaled targets
    x, t = F.net_inputs(tr, "regressor", [0, 5, 43877], (0, 0, 0), 64, T.SDF, 3.0)
    assert np.allclose(x, (tr["ijk"][[0, 5, 43877]] + 0.5) / 64)
    assert np.allclose(t, tr["values"][[0, 5, 43877]] / 3.0)
    assert np.all(np.abs(t) <= 1.0)
    # level-0 slots of active voxels are labelled 1, and the labels sum to N
    slots = np.arange(F.population(tr, "l0"))
    _, lab = F.net_inputs(tr, "l0", slots, (0, 0, 0), 64, T.SDF, 3.0)
    assert lab.sum() == len(tr["values"])
    s = tr["vox_leaf"] * 512 + tr["vox_n0"]
    assert np.all(lab[s] == 1)
    x, _ = F.net_inputs(tr, "l0", s[:10], (0, 0, 0), 64, T.SDF, 3.0)
    assert np.allclose(x, (tr["ijk"][:10] + 0.5) / 64)
    # level-1 slots: one class-0 label per leaf, the rest inactive tiles
    slots = np.arange(F.population(tr, "l1"))
    x, c = F.net_inputs(tr, "l1", slots, (0, 0, 0), 64, T.SDF, 3.0)
    assert (c == 0).sum() == len(tr["leaf_origin"]) and (c == 1).sum() == 0
    assert np.allclose(x[0], [4 / 64, 4 / 64, 4 / 64])


def test_fit_lowers_loss(sphere):
    shapes = mlp.layer_shapes(36, 64, 3, 1)
    th0 = workloads.init_params(36, 64, 3, 1, seed=0).astype(np.float64)
    B = mlp.pe_matrix(6)
    th, m, v, losses = F.train(th0, shapes, B, sphere, "regressor", (0, 0, 0), 64, T.SDF, 3.0,
                               steps=100, batch=1024, seed=0, lr0=1e-3)
    assert losses[-5:].mean() < 0.25 * losses[:3].mean()
    _, _, _, lc = F.train(th0, shapes, B, sphere, "l0", (0, 0, 0), 64, T.SDF, 3.0,
                          steps=100, batch=1024, seed=0, lr0=1e-3)
    assert lc[-5:].mean() < 0.85 * lc[:3].mean()


def test_train_resume_is_exact(sphere):
    shapes = mlp.layer_shapes(36, 64, 3, 1)
    th0 = workloads.init_params(36, 64, 3, 1, seed=1).astype(np.float64)
    B = mlp.pe_matrix(6)
    a = F.train(th0, shapes, B, sphere, "regressor", (0, 0, 0), 64, T.SDF, 3.0, steps=6, batch=256)
    b1 = F.train(th0, shapes, B, sphere, "regressor", (0, 0, 0), 64, T.SDF, 3.0, steps=3, batch=256)
    b2 = F.train(b1[0], shapes, B, sphere, "regressor", (0, 0, 0), 64, T.SDF, 3.0, steps=3, batch=256,
                 step0=3, m0=b1[1], v0=b1[2])
    assert np.array_equal(a[0], b2[0])


def test_errors_known_cases(sphere):
    tr = sphere
    rep = F.errors(tr, tr["values"].copy(), T.SDF, pred_mask=tr["leaf_mask"].copy())
    assert rep["max_abs"] == 0.0 and rep["rms"] == 0.0 and rep["iou"] == 1.0
    assert rep["fp"] == 0 and rep["fn"] == 0
    vh = tr["values"].copy(); vh[7] += 0.5; vh[9] -= 2.0
    pm = tr["leaf_mask"].copy()
    pm[0, 0] ^= np.uint64(0b101)    # flip two slots of leaf 0
    rep = F.errors(tr, vh, T.SDF, pred_mask=pm)
    assert rep["max_abs"] == 2.0
    assert np.isclose(rep["rms"], np.sqrt((0.25 + 4.0) / len(vh)))
    truth = [(int(tr["leaf_mask"][0, 0]) >> b) & 1 for b in (0, 2)]
    assert rep["fp"] == truth.count(0) and rep["fn"] == truth.count(1)


def test_mask_from_logits_and_classes():
    logits = -np.ones(2 * 512); logits[[0, 63, 64, 511, 512 + 100]] = 1.0
    w = F.mask_from_logits(logits, 2)
    assert int(w[0, 0]) == 1 | (1 << 63) and int(w[0, 1]) == 1 and int(w[0, 7]) == 1 << 63
    assert int(w[1, 1]) == 1 << 36
    assert F.l1_classes(np.array([[1.0, 1.0, 0.0], [0.0, 2.0, 2.0], [0, 0, 3.0]])).tolist() == [0, 1, 2]


# ---------------------------------------------------------------- warm-start sequence (Sec. 3.6)
_SEQ_SHAPES = mlp.layer_shapes(36, 16, 2, 1)
_SEQ_B = mlp.pe_matrix(6)


def _seq_frames(centers, radius=20.0):
    out = []
    for c in centers:
        v = workloads.sphere_sdf(center=c, radius=radius).numpy()
        ijk, vals = T.active_set_dense(v, (0, 0, 0), T.SDF, 3.0)
        out.append(T.build(ijk, vals))
    return out


def _sched(steps, lr, seed, batch=256):
    return dict(steps=steps, batch=batch, seed=seed, lr=lr, lr_decay=0.975, lr_interval=100)


def test_sequence_single_frame_is_cold_then_refit(sphere):
    th0 = workloads.init_params(36, 16, 2, 1, seed=3).astype(np.float64)
    cold, warm = _sched(6, 1e-2, 5), _sched(4, 1e-3, 9)
    ths, runs, L = F.train_sequence(th0, _SEQ_SHAPES, _SEQ_B, [sphere], "regressor", (0, 0, 0), 64, T.SDF, 3.0,
                                    cold, warm)
    a, _, _, La = F.train(th0, _SEQ_SHAPES, _SEQ_B, sphere, "regressor", (0, 0, 0), 64, T.SDF, 3.0, 6, 256,
                          seed=5, lr0=1e-2)
    # the refit starts from a fresh Adam state: its first update is -lr g / (|g| + eps)
    b, _, _, Lb = F.train(a, _SEQ_SHAPES, _SEQ_B, sphere, "regressor", (0, 0, 0), 64, T.SDF, 3.0, 1, 256,
                          seed=9, lr0=1e-3)
    g = F.step_grad(a, _SEQ_SHAPES, _SEQ_B,
                    *F.net_inputs(sphere, "regressor", F.sampler.iid_indices(9, F.NET_STREAM["regressor"], 0, 256,
                                                                             len(sphere["values"])),
                                  (0, 0, 0), 64, T.SDF, 3.0), "regressor")[1]
    assert np.allclose(b - a, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
    assert runs == [10]
    assert np.allclose(L[0][:6], La, rtol=0, atol=0)
    assert L[0][6] == Lb[0]


def test_sequence_stop_rule_brute_force():
    """With a zero warm rate the weights never move after frame 0, so every
    frame's batch losses are losses of one fixed network; the number of steps a
    frame runs must be one past the first batch whose loss is below frame 0's
    final loss (or the cap), found here by evaluating the batches directly."""
    frames = _seq_frames([(32.0, 32.0, 32.0), (32.5, 32.0, 31.5), (33.0, 32.0, 31.0)])
    th0 = workloads.init_params(36, 16, 2, 1, seed=4).astype(np.float64)
    cold, warm = _sched(40, 1e-2, 1), _sched(12, 0.0, 7)
    ths, runs, L = F.train_sequence(th0, _SEQ_SHAPES, _SEQ_B, frames, "regressor", (0, 0, 0), 64, T.SDF, 3.0,
                                    cold, warm)
    target = L[0][-1]
    params = mlp.unflatten(ths[0], _SEQ_SHAPES)
    for f in (1, 2):
        assert np.array_equal(ths[f], ths[0])
        tr = frames[f]
        batch_losses = []
        for j in range(12):
            idx = F.sampler.iid_indices(7 + f, F.NET_STREAM["regressor"], j, 256, len(tr["values"]))
            x = (tr["ijk"][idx] + 0.5) / 64.0
            t = tr["values"][idx] / 3.0
            y, _ = mlp.forward(params, mlp.encode(x, _SEQ_B))
            batch_losses.append(np.mean((y[:, 0] - t) ** 2))
        below = [j for j, l in enumerate(batch_losses) if l < target]
        expect = below[0] + 1 if below else 12
        assert runs[f] == expect
        assert np.allclose(L[f], batch_losses[:expect], rtol=1e-12, atol=0)
    assert min(runs[1:]) < 12, "the case should exercise an early stop"


def test_sequence_warm_start_needs_fewer_steps():
    """The point of the warm start: later frames of a slowly moving sphere reach
    frame 0's final loss within the cap, well before a cold fit would."""
    frames = _seq_frames([(32.0, 32.0, 32.0), (32.25, 32.0, 32.0), (32.5, 32.0, 32.0)])
    th0 = workloads.init_params(36, 16, 2, 1, seed=4).astype(np.float64)
    cold, warm = _sched(60, 1e-2, 1), _sched(30, 1e-3, 7)
    ths, runs, L = F.train_sequence(th0, _SEQ_SHAPES, _SEQ_B, frames, "regressor", (0, 0, 0), 64, T.SDF, 3.0,
                                    cold, warm)
    assert runs[0] == 90
    assert all(r < 30 for r in runs[1:]), runs
    assert all(l[-1] < L[0][-1] for l in L[1:])


def test_errors_l1_counts(sphere):
    """Level-1 report: the truth has exactly one child-leaf slot per leaf; a
    perfect prediction has no errors; planted mistakes are counted exactly."""
    tr = sphere
    n = 4096 * len(tr["l1_origin"])
    _, truth = F.net_inputs(tr, "l1", np.arange(n), (0, 0, 0), 64, T.SDF, 3.0)
    assert int(np.sum(truth == 0)) == len(tr["leaf_origin"])
    rep = F.errors_l1(tr, truth)
    assert rep == dict(n_slots=n, fp=0, fn=0, mismatch=0)
    c = truth.copy()
    child = np.nonzero(truth == 0)[0]
    other = np.nonzero(truth == 2)[0]
    c[child[:3]] = 2          # 3 false negatives
    c[other[:5]] = 0          # 5 false positives
    c[other[5:7]] = 1         # 2 plain mismatches
    assert F.errors_l1(tr, c) == dict(n_slots=n, fp=5, fn=3, mismatch=10)


def test_topology_from_true_decisions_is_the_tree(sphere):
    """Rebuilding the lower levels from the true classes, masks and values gives
    back the tree exactly; planted voxel mistakes are counted exactly."""
    tr = sphere
    n = 4096 * len(tr["l1_origin"])
    _, truth = F.net_inputs(tr, "l1", np.arange(n), (0, 0, 0), 64, T.SDF, 3.0)
    keys = set(map(tuple, tr["ijk"].tolist()))
    lut = {k: v for k, v in zip(map(tuple, tr["ijk"].tolist()), tr["values"])}
    active = lambda p: np.array([tuple(q) in keys for q in p.tolist()])
    values = lambda p, a: np.array([lut[tuple(q)] for q in p[a].tolist()])
    pred = F.topology_from_decisions(tr, truth, active, values)
    assert np.array_equal(pred["leaf_origin"], tr["leaf_origin"])
    assert np.array_equal(pred["ijk"], tr["ijk"]) and np.array_equal(pred["values"], tr["values"])
    rep = F.errors_topology(tr["ijk"], tr["values"], pred["ijk"], pred["values"])
    assert rep == dict(n_true=len(tr["values"]), n_pred=len(tr["values"]), fp=0, fn=0, n_common=len(tr["values"]),
                       max_abs=0.0, rms=0.0)
    # drop 5 voxels, add 3 outside the band, perturb one value by 0.5
    ijk = np.concatenate([pred["ijk"][5:], [[0, 0, 0], [0, 0, 1], [1, 0, 0]]])
    val = np.concatenate([pred["values"][5:], [9.0, 9.0, 9.0]])
    val[0] += 0.5
    rep = F.errors_topology(tr["ijk"], tr["values"], ijk, val)
    N = len(tr["values"])
    assert (rep["n_pred"], rep["fp"], rep["fn"], rep["n_common"]) == (N - 2, 3, 5, N - 5)
    assert rep["max_abs"] == 0.5 and np.isclose(rep["rms"], np.sqrt(0.25 / (N - 5)))


def test_query_random_access_pins():
    """Random access (Sec. 3.5): queries at active voxel centres reproduce the
    decode of those voxels; the hit set equals a brute-force walk over leaf
    origins and masks; misses (outside every leaf, inactive voxels inside a
    leaf, non-finite positions) get the background value."""
    import workloads
    v = workloads.sphere_sdf(n=24, center=(12.0, 12.0, 12.0), radius=7.0).numpy()
    ijk, vals = T.active_set_dense(v, (-5, 3, 0), T.SDF, 2.0)
    tr = T.build(ijk, vals)
    shapes = mlp.layer_shapes(36, 16, 2, 1)
    th = np.random.default_rng(0).uniform(-0.5, 0.5, mlp.param_count(36, 16, 2, 1))
    B = mlp.pe_matrix(6)
    lo, D = (-5, 3, 0), 24
    idx = np.arange(0, len(vals), 7)
    qc = tr["ijk"][idx].astype(np.float64) + 0.5
    vq, hq = F.query_values(th, shapes, B, tr, lo, D, T.SDF, 2.0, qc, background=9.0)
    assert hq.all()
    assert np.array_equal(vq, F.decode_values(th, shapes, B, tr, lo, D, T.SDF, 2.0, idx=idx))
    rng = np.random.default_rng(1)
    q = rng.uniform(-8.0, 30.0, (3000, 3))
    q[:5] = [[np.nan, 0, 0], [np.inf, 1, 1], [0.0, 0.0, -np.inf], [1e12, 0, 0], [-3e9, 5, 5]]
    hits = F.query_hits(tr, q)
    # brute force: leaf lookup by origin, then the mask bit
    leaves = {tuple(o): i for i, o in enumerate(np.asarray(tr["leaf_origin"], np.int64).tolist())}
    want = np.zeros(len(q), bool)
    for i, p in enumerate(q):
        if not np.all(np.isfinite(p)) or np.any(np.abs(p) >= 2.0 ** 31 - 2):
            continue
        c = np.floor(p).astype(np.int64)
        li = leaves.get(tuple(c & ~7))
        if li is None:
            continue
        n0 = int(((c[0] & 7) << 6) | ((c[1] & 7) << 3) | (c[2] & 7))
        want[i] = bool((int(tr["leaf_mask"][li, n0 >> 6]) >> (n0 & 63)) & 1)
    assert np.array_equal(hits, want) and 0 < hits.sum() < len(q)
    vq, hq = F.query_values(th, shapes, B, tr, lo, D, T.SDF, 2.0, q, background=9.0)
    assert np.array_equal(hq, hits) and np.all(vq[~hits] == 9.0) and np.all(np.abs(vq[hits]) < 9.0)


def test_topology_patches_restore_the_active_set():
    """Patches: brute-force set differences, canonical order (that of the tree
    build), and pred - fp + fn equals the true active set."""
    rng = np.random.default_rng(3)
    truth = np.unique(rng.integers(-20, 20, (400, 3)), axis=0)
    keep = rng.random(len(truth)) < 0.8
    extra = np.unique(rng.integers(-20, 20, (120, 3)), axis=0)
    pred = np.unique(np.concatenate([truth[keep], extra]), axis=0)
    fp, fn = F.topology_patches(truth, pred)
    ts, ps = set(map(tuple, truth.tolist())), set(map(tuple, pred.tolist()))
    assert set(map(tuple, fp.tolist())) == ps - ts and len(fp) == len(ps - ts)
    assert set(map(tuple, fn.tolist())) == ts - ps and len(fn) == len(ts - ps)
    assert len(fp) > 0 and len(fn) > 0
    assert np.array_equal(fp, T.build(fp, np.zeros(len(fp)))["ijk"])
    assert (ps - set(map(tuple, fp.tolist()))) | set(map(tuple, fn.tolist())) == ts
    e, f = F.topology_patches(truth, truth)
    assert len(e) == 0 and len(f) == 0


# ---------------------------------------------------------------- IoU and the decided topology (Sec. 4, 3.3, 3.5)
def test_iou_planted_case():
    """IoU of the interiors {v <= 0} (Sec. 4) on six hand-counted voxels, zeros
    included: truth interior {0, 1, 4, 5}, decoded interior {0, 2, 3, 4, 5};
    intersection {0, 4, 5} = 3, union = all six, IoU = 1/2.  The readings v < 0
    (2/3) or intersection over the true interior (3/4) give other values."""
    ijk = np.array([[0, 0, 0], [0, 0, 1], [0, 1, 0], [1, 0, 0], [9, 0, 0], [0, 9, 9]], np.int32)
    truth = np.array([-1.0, 0.0, 0.5, 2.0, -0.2, 0.0])
    tr = T.build(ijk, truth)
    order = {tuple(p): i for i, p in enumerate(ijk.tolist())}
    perm = np.array([order[tuple(p)] for p in tr["ijk"].tolist()])  # canonical voxel order -> planted index
    decoded = np.array([-0.5, 0.1, -0.1, 0.0, -1.0, 0.0])[perm]
    rep = F.errors(tr, decoded, T.SDF)
    assert rep["iou"] == 0.5
    # a decode that keeps every interior voxel and adds none is exact
    assert F.errors(tr, truth[perm], T.SDF)["iou"] == 1.0
    # fog volumes carry no IoU (RMSE is their measure)
    assert "iou" not in F.errors(tr, decoded, T.FOG)


def _true_classes(tr):
    n = 4096 * len(tr["l1_origin"])
    slots = np.arange(n)
    child = T.mask_bits(tr["l1_child"], slots >> 12, slots & 4095)
    return np.where(child == 1, 0, 2)


def test_topology_active_rule_rebuilds_truth_sdf():
    """With the true level-1 classes and a regressor that returns the exact level
    set, the active rule |v| <= band rebuilds the true active set and values.
    The sphere has lattice voxels at |v| = 3 exactly (distance 27 or 21 from the
    centre), so a strict band would drop them."""
    grid = workloads.sphere_sdf().numpy().astype(np.float64)
    ijk, vals = T.active_set_dense(grid, (0, 0, 0), T.SDF, 3.0)
    tr = T.build(ijk, vals)
    assert np.sum(np.abs(tr["values"]) == 3.0) > 0

    def sdf(p):
        return np.linalg.norm(np.asarray(p, np.float64) - 32.0, axis=1) - 24.0

    out = F.topology_from_values(tr, _true_classes(tr), T.SDF, 3.0, sdf)
    assert np.array_equal(out["ijk"], tr["ijk"])
    assert np.allclose(out["values"], tr["values"], rtol=0, atol=4e-6)  # the grid holds float32 values
    assert np.array_equal(out["leaf_origin"], tr["leaf_origin"])
    # a level-0 decision that returns the true mask gives the same tree
    act = {tuple(p) for p in tr["ijk"].tolist()}
    out0 = F.topology_from_values(tr, _true_classes(tr), T.SDF, 3.0, sdf,
                                  active_fn=lambda p: np.array([tuple(q) in act for q in p.tolist()]))
    assert np.array_equal(out0["ijk"], tr["ijk"]) and np.allclose(out0["values"], tr["values"], rtol=0, atol=4e-6)


def test_topology_active_rule_rebuilds_truth_fog():
    """Fog keeps v > threshold (strict): planted voxels at exactly the threshold
    stay inactive, and a regressor returning the grid rebuilds the true set."""
    rng = np.random.default_rng(3)
    grid = rng.random((24, 20, 16))
    grid[grid < 0.6] = 0.0
    grid[3, 4, 5] = grid[10, 11, 12] = grid[20, 1, 2] = 0.5      # exactly the threshold
    origin = (-8, 0, 16)
    ijk, vals = T.active_set_dense(grid, origin, T.FOG, 0.5)
    tr = T.build(ijk, vals)

    def lookup(p):
        q = np.asarray(p, np.int64) - np.asarray(origin)
        inside = np.all((q >= 0) & (q < np.array(grid.shape)), axis=1)
        v = np.zeros(len(q))
        v[inside] = grid[q[inside, 0], q[inside, 1], q[inside, 2]]
        return v

    out = F.topology_from_values(tr, _true_classes(tr), T.FOG, 0.5, lookup)
    assert np.array_equal(out["ijk"], tr["ijk"]) and np.array_equal(out["values"], tr["values"])
    assert not any(tuple(p) in {(-5, 4, 21), (2, 11, 28), (12, 1, 18)} for p in out["ijk"].tolist())
    # a level-1 class that drops a leaf drops exactly that leaf's voxels
    cls = _true_classes(tr)
    first_leaf = np.nonzero(cls == 0)[0][0]
    cls[first_leaf] = 2
    out2 = F.topology_from_values(tr, cls, T.FOG, 0.5, lookup)
    assert len(out2["ijk"]) == len(tr["ijk"]) - int(np.sum(tr["vox_leaf"] == 0))


# ---------------------------------------------------------------- active tiles (Sec. 3.3.1)
@pytest.fixture(scope="module")
def fog_tiles():
    v = workloads.saturated_fog().numpy()
    ijk, vals = T.active_set_dense(v, (0, 0, 0), T.FOG, 0.05)
    return T.prune_tiles(T.build(ijk, vals))


def test_tile_samples_are_the_active_tile_slots(fog_tiles):
    """The tile regressor's samples are the level-1 slots whose ternary class is
    'active tile', at the same leaf centres the level-1 classifier sees, with the
    tile value (fog: unscaled) as target."""
    tr = fog_tiles
    nt = F.population(tr, "tile")
    assert nt == len(tr["tile_value"]) >= 4
    key = tr["tile_l1"] * 4096 + tr["tile_n1"]
    x1, c1 = F.net_inputs(tr, "l1", key, (0, 0, 0), 64, T.FOG, 0.05)
    xt, tt = F.net_inputs(tr, "tile", np.arange(nt), (0, 0, 0), 64, T.FOG, 0.05)
    assert np.array_equal(x1, xt) and np.all(c1 == 1)
    assert np.all(tt == 1.0) and np.array_equal(tt, tr["tile_value"])
    assert np.allclose(xt, (tr["tile_origin"] + 4) / 64)
    _, call = F.net_inputs(tr, "l1", np.arange(F.population(tr, "l1")), (0, 0, 0), 64, T.FOG, 0.05)
    assert (call == 1).sum() == nt and (call == 0).sum() == len(tr["leaf_origin"])


def test_topology_with_tiles_from_true_decisions(fog_tiles):
    """The top-down decode with the true ternary classes, masks, values and tile
    values rebuilds the voxels and the tiles exactly; a tile predicted inactive
    is missing from the result, and planted tile errors are measured exactly."""
    tr = fog_tiles
    n = 4096 * len(tr["l1_origin"])
    _, cls = F.net_inputs(tr, "l1", np.arange(n), (0, 0, 0), 64, T.FOG, 0.05)
    keys = set(map(tuple, tr["ijk"].tolist()))
    lut = {k: v for k, v in zip(map(tuple, tr["ijk"].tolist()), tr["values"])}
    tlut = {tuple(o): v for o, v in zip(tr["tile_origin"].tolist(), tr["tile_value"])}
    active = lambda p: np.array([tuple(q) in keys for q in p.tolist()])
    values = lambda p, a: np.array([lut[tuple(q)] for q in p[a].tolist()])
    tiles = lambda o: np.array([tlut[tuple(q)] for q in o.tolist()])
    pred = F.topology_from_decisions(tr, cls, active, values, tiles)
    assert np.array_equal(pred["ijk"], tr["ijk"]) and np.array_equal(pred["values"], tr["values"])
    assert np.array_equal(pred["tile_key"], tr["tile_l1"] * 4096 + tr["tile_n1"])
    assert np.array_equal(pred["tile_origin"], tr["tile_origin"])
    assert np.array_equal(pred["tile_value"], tr["tile_value"])
    # without a tile regressor no tiles come out
    assert len(F.topology_from_decisions(tr, cls, active, values)["tile_key"]) == 0
    # the first tile predicted as an inactive tile
    cls2 = cls.copy()
    cls2[pred["tile_key"][0]] = 2
    pred2 = F.topology_from_decisions(tr, cls2, active, values, tiles)
    assert np.array_equal(pred2["tile_key"], pred["tile_key"][1:])
    # planted tile value errors
    that = tr["tile_value"].copy()
    that[1] += 0.25
    that[2] -= 0.125
    rep = F.errors_tiles(tr, that)
    assert rep["n"] == len(that) and rep["max_abs"] == 0.25
    assert np.isclose(rep["rms"], np.sqrt((0.0625 + 0.015625) / len(that)))


def test_query_tiles_pins(fog_tiles):
    """Random access through the tiles: queries anywhere inside an active tile's
    8^3 region find it (brute force over the tile origins), queries in leaves,
    outside the level-1 nodes or non-finite find none; with a tile regressor such
    queries return the tile decode's value, every voxel hit the regressor's."""
    tr = fog_tiles
    rng = np.random.default_rng(5)
    t_pick = rng.integers(0, len(tr["tile_value"]), 200)
    q_in = tr["tile_origin"][t_pick] + rng.uniform(0.0, 8.0, (200, 3))
    q_rand = rng.uniform(-10.0, 80.0, (2000, 3))
    q = np.concatenate([q_in, q_rand, [[np.nan, 1, 1], [1e12, 0, 0]]])
    got = F.query_tiles(tr, q)
    assert np.array_equal(got[:200], t_pick)
    origins = [tuple(o) for o in tr["tile_origin"].tolist()]
    for i in range(200, len(q)):
        if not np.all(np.isfinite(q[i])) or np.any(np.abs(q[i]) >= 2.0 ** 31 - 2):
            assert got[i] == -1
            continue
        o = tuple(int(c) & ~7 for c in np.floor(q[i]))
        assert got[i] == (origins.index(o) if o in origins else -1)
    hits = F.query_hits(tr, q)
    assert not np.any(hits & (got >= 0)) and hits.sum() > 0 and (got >= 0).sum() > 200
    shapes = mlp.layer_shapes(36, 16, 2, 1)
    th = np.random.default_rng(0).uniform(-0.5, 0.5, mlp.param_count(36, 16, 2, 1))
    tt = np.random.default_rng(1).uniform(-0.5, 0.5, mlp.param_count(36, 16, 2, 1))
    B = mlp.pe_matrix(6)
    v, h = F.query_values(th, shapes, B, tr, (0, 0, 0), 64, T.FOG, 0.05, q, background=-1.0,
                          tile=(tt, shapes, B))
    vt = F.decode_tiles(tt, shapes, B, tr, (0, 0, 0), 64, T.FOG, 0.05)
    assert np.array_equal(v[got >= 0], vt[got[got >= 0]])
    v0, _ = F.query_values(th, shapes, B, tr, (0, 0, 0), 64, T.FOG, 0.05, q, background=-1.0)
    assert np.array_equal(v[~(got >= 0)], v0[~(got >= 0)]) and np.all(v0[got >= 0] == -1.0)
