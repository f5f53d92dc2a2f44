"""Encode (fit) and decode of NeuralVDB's lower tree levels (oracle).

Encoding trains each network on its own samples (Sec. 3.2.1, 3.3.1):
  * voxel-value regressor: active voxels only, target v/band for a
    narrow-band SDF (scaled into [-1,1]) and v for a fog volume (Sec. 3.2);
  * level-0 mask classifier: every voxel slot of the existing leaves
    ("performed within level-1's children nodes"), label = active bit;
  * level-1 node classifier: every leaf slot of the existing level-1 nodes at
    the leaf centre, label = child (0) / active tile (1) / inactive tile (2);
  * tile value regressor: the active tiles at their leaf-slot centres, target
    scaled as the voxel regressor's (Sec. 3.3.1).
Decoding (Sec. 3.5, offline sequential access) evaluates the networks over all
slots: mask bit = logit > 0, node class = argmax with ties to the lowest index,
value = y * band (SDF) or y (fog).  The error report follows the quality
measures of Sec. 4 (IoU of the interior for level sets, RMSE for fog) plus max
error and the classifier false positives / negatives.
"""
import numpy as np

from . import fp8 as fp8_form, mlp, sampler, tree as T

NET_STREAM = {"regressor": sampler.STREAM_REGRESSOR, "l0": sampler.STREAM_L0, "l1": sampler.STREAM_L1,
              "tile": sampler.STREAM_TILE}
NET_LOSS = {"regressor": "mse", "l0": "bce", "l1": "ce", "tile": "mse"}


def population(tr, net):
    if net == "regressor":
        return len(tr["values"])
    if net == "l0":
        return 512 * len(tr["leaf_origin"])
    if net == "l1":
        return 4096 * len(tr["l1_origin"])
    if net == "tile":
        return len(tr["tile_value"])
    raise ValueError(net)


def net_inputs(tr, net, idx, lo, D, kind, band):
    """Normalised coordinates and targets of samples idx of network `net`."""
    idx = np.asarray(idx, dtype=np.int64)
    if net == "regressor":
        x = mlp.normalize_voxel(tr["ijk"][idx], lo, D)
        v = tr["values"][idx]
        t = v / band if kind == T.SDF else v
    elif net == "l0":
        leaf, n0 = idx >> 9, idx & 511
        p = tr["leaf_origin"][leaf].astype(np.int64) + T.n0_to_offset(n0)
        x = mlp.normalize_voxel(p, lo, D)
        t = T.mask_bits(tr["leaf_mask"], leaf, n0).astype(np.float64)
    elif net == "l1":
        node, n1 = idx >> 12, idx & 4095
        o = tr["l1_origin"][node].astype(np.int64) + T.n1_to_offset(n1)
        x = mlp.normalize_leaf_slot(o, lo, D)
        child = T.mask_bits(tr["l1_child"], node, n1)
        active = T.mask_bits(tr["l1_active"], node, n1)
        t = np.where(child == 1, 0, np.where(active == 1, 1, 2))
    elif net == "tile":
        o = tr["l1_origin"][tr["tile_l1"][idx]].astype(np.int64) + T.n1_to_offset(tr["tile_n1"][idx])
        x = mlp.normalize_leaf_slot(o, lo, D)
        v = tr["tile_value"][idx]
        t = v / band if kind == T.SDF else v
    else:
        raise ValueError(net)
    return x, t


def step_grad(theta, shapes, B, x, t, net):
    """Loss and flat gradient of one batch."""
    params = mlp.unflatten(theta, shapes)
    y, cache = mlp.forward(params, mlp.encode(x, B))
    kind = NET_LOSS[net]
    gy = mlp.output_grad(kind, y, t)
    return mlp.loss(kind, y, t), mlp.flatten(mlp.backward(params, cache, gy))


def param_grad(theta, shapes, B, x, gy):
    """Gradient of sum(gy * f(x)) with respect to the parameters (vector-Jacobian product)."""
    params = mlp.unflatten(theta, shapes)
    _, cache = mlp.forward(params, mlp.encode(x, B))
    return mlp.flatten(mlp.backward(params, cache, np.asarray(gy, np.float64).reshape(len(x), -1)))


def train(theta0, shapes, B, tr, net, lo, D, kind, band, steps, batch, seed=0, lr0=1e-3,
          decay=0.975, interval=100, idx_batches=None, step0=0, m0=None, v0=None, stop_below=None):
    """Adam fit of one network.  Batch indices come from the SplitMix64 sampler
    (stream of the network, step counted from step0) unless idx_batches is given.
    With stop_below, no further step is taken once a step's batch loss is below
    it (the warm-start stopping rule of Sec. 3.6); the returned losses then hold
    only the steps that ran."""
    theta = np.array(theta0, dtype=np.float64)
    m = np.zeros_like(theta) if m0 is None else np.array(m0, np.float64)
    v = np.zeros_like(theta) if v0 is None else np.array(v0, np.float64)
    pop = population(tr, net)
    losses = []
    for k in range(steps):
        if stop_below is not None and losses and losses[-1] < stop_below:
            break
        s = step0 + k + 1
        if idx_batches is not None:
            idx = idx_batches[k]
        else:
            idx = sampler.iid_indices(seed, NET_STREAM[net], s - 1, batch, pop)
        x, t = net_inputs(tr, net, idx, lo, D, kind, band)
        L, g = step_grad(theta, shapes, B, x, t, net)
        losses.append(L)
        theta, m, v = mlp.adam_step(theta, g, m, v, s, mlp.lr_at(s, lr0, decay, interval))
    return theta, m, v, np.array(losses)


def train_sequence(theta0, shapes, B, frames, net, lo, D, kind, band, cold, warm):
    """Warm-start encoder of an animated sequence (Sec. 3.6) for one network.

    Frame 0 is fitted twice from theta0: `cold` (the target learning rate), then
    `warm` (the smaller refinement rate).  The final batch loss of that second
    pass is the target every later frame aims for: frame f >= 1 starts from the
    weights of frame f-1 and runs up to warm['steps'] steps, stopping as soon as
    a step's loss is below the target.  Each pass has its own Adam state (zero
    moments, step count from 1); pass seeds are cold['seed'] for the first pass
    and warm['seed'] + f for frame f's warm pass.
    cold / warm: dicts with steps, batch, seed, lr, lr_decay, lr_interval.
    Returns (thetas per frame, steps run per frame, losses per frame)."""
    def run(theta, tree, d, seed, stop):
        th, _, _, L = train(theta, shapes, B, tree, net, lo, D, kind, band, d["steps"], d["batch"], seed=seed,
                            lr0=d["lr"], decay=d["lr_decay"], interval=d["lr_interval"], stop_below=stop)
        return th, L
    th, La = run(theta0, frames[0], cold, cold["seed"], None)
    th, Lb = run(th, frames[0], warm, warm["seed"], None)
    target = Lb[-1]
    thetas, runs, losses = [th], [len(La) + len(Lb)], [np.concatenate([La, Lb])]
    for f in range(1, len(frames)):
        th, L = run(th, frames[f], warm, warm["seed"] + f, target)
        thetas.append(th)
        runs.append(len(L))
        losses.append(L)
    return thetas, runs, losses


def _batched_predict(theta, shapes, B, x, chunk=1 << 15, fp8=False):
    params = mlp.unflatten(theta, shapes)
    out = []
    for i in range(0, len(x), chunk):
        z0 = mlp.encode(x[i:i + chunk], B)
        y = fp8_form.forward_fp8(params, z0) if fp8 else mlp.forward(params, z0)[0]
        out.append(y)
    return np.concatenate(out) if out else np.zeros((0, shapes[-1][0]))


def decode_values(theta, shapes, B, tr, lo, D, kind, band, idx=None, fp8=False):
    """Regressor decode at the true active voxels (all, or the subset idx); fp8
    selects the FP8 form of the forward pass."""
    idx = np.arange(len(tr["values"])) if idx is None else np.asarray(idx)
    x = mlp.normalize_voxel(tr["ijk"][idx], lo, D)
    y = _batched_predict(theta, shapes, B, x, fp8=fp8)[:, 0]
    return y * band if kind == T.SDF else y


def decode_l0(theta, shapes, B, tr, lo, D, slots=None, fp8=False):
    """Level-0 classifier logits at leaf slots (all 512 L, or the subset `slots`)."""
    slots = np.arange(population(tr, "l0")) if slots is None else np.asarray(slots)
    x, _ = net_inputs(tr, "l0", slots, lo, D, T.SDF, 1.0)
    return _batched_predict(theta, shapes, B, x, fp8=fp8)[:, 0]


def decode_l1(theta, shapes, B, tr, lo, D, slots=None, fp8=False):
    """Level-1 classifier logits at leaf slots of the L1 nodes."""
    slots = np.arange(population(tr, "l1")) if slots is None else np.asarray(slots)
    x, _ = net_inputs(tr, "l1", slots, lo, D, T.SDF, 1.0)
    return _batched_predict(theta, shapes, B, x, fp8=fp8)


def decode_tiles(theta, shapes, B, tr, lo, D, kind, band, fp8=False):
    """Tile value regressor at every active tile of the tree, in value units."""
    x, _ = net_inputs(tr, "tile", np.arange(len(tr["tile_value"])), lo, D, kind, band)
    y = _batched_predict(theta, shapes, B, x, fp8=fp8)[:, 0]
    return y * band if kind == T.SDF else y


def errors_tiles(tr, that):
    """max |t^ - t| and RMS over the active tiles of the tree (value units)."""
    d = np.asarray(that, np.float64) - tr["tile_value"]
    return dict(n=len(d), max_abs=float(np.max(np.abs(d))) if len(d) else 0.0,
                rms=float(np.sqrt(np.mean(d * d))) if len(d) else 0.0)


def mask_from_logits(logits, n_leaves):
    """Predicted leaf masks (L, 8) uint64 from slot logits in leaf-major order."""
    bits = (np.asarray(logits).reshape(n_leaves, 512) > 0)
    words = np.zeros((n_leaves, 8), dtype=np.uint64)
    for n in range(512):          # bit n -> word n >> 6, position n & 63
        words[:, n >> 6] |= bits[:, n].astype(np.uint64) << np.uint64(n & 63)
    return words


def l1_classes(logits):
    """argmax over the three classes, ties resolved to the lowest index."""
    return np.argmax(np.asarray(logits), axis=1)


def errors_l1(tr, classes):
    """Level-1 classifier report over every leaf slot of the level-1 nodes:
    false positives (predicted child leaf, none there), false negatives (child
    leaf predicted as a tile) and class mismatches."""
    n = 4096 * len(tr["l1_origin"])
    _, truth = net_inputs(tr, "l1", np.arange(n), (0, 0, 0), 1, T.SDF, 1.0)
    truth = truth.astype(np.int64)
    c = np.asarray(classes, np.int64).reshape(-1)
    return dict(n_slots=n, fp=int(np.sum((c == 0) & (truth != 0))), fn=int(np.sum((c != 0) & (truth == 0))),
                mismatch=int(np.sum(c != truth)))


def topology_from_decisions(tr, classes, active_fn, value_fn, tile_fn=None):
    """Lower tree levels rebuilt from per-slot decisions (Sec. 3.3, 3.5).

    classes: level-1 class of every leaf slot of tr's level-1 nodes (0 = leaf,
    1 = active tile); active_fn(p) -> bool per voxel coordinate of the predicted
    leaves' slots; value_fn(p, active) -> values of the active voxels;
    tile_fn(o) -> values of the predicted active tiles at leaf origins o (the top-
    down traversal of Sec. 3.3.1: an active tile takes the tile regressor's value
    and has no leaf below it).  Returns the predicted leaf origins, voxel
    coordinates and values in canonical order, and the predicted tiles as keys
    (level-1 node << 12 | n1), origins and values (empty without tile_fn)."""
    flat = np.asarray(classes).reshape(-1)
    tslots = np.nonzero(flat == 1)[0] if tile_fn is not None else np.zeros(0, np.int64)
    tile_o = tr["l1_origin"][tslots >> 12].astype(np.int64) + T.n1_to_offset(tslots & 4095)
    tile_v = np.asarray(tile_fn(tile_o), np.float64) if len(tslots) else np.zeros(0)
    slots = np.nonzero(flat == 0)[0]
    node, n1 = slots >> 12, slots & 4095
    leaf_o = tr["l1_origin"][node].astype(np.int64) + T.n1_to_offset(n1)
    p = (leaf_o[:, None, :] + T.n0_to_offset(np.arange(512))[None, :, :]).reshape(-1, 3)
    act = np.asarray(active_fn(p), bool) if len(p) else np.zeros(0, bool)
    ijk = p[act]
    values = np.asarray(value_fn(p, act), np.float64) if len(ijk) else np.zeros(0)
    return dict(leaf_origin=leaf_o, ijk=ijk, values=values, tile_key=tslots.astype(np.int64), tile_origin=tile_o,
                tile_value=tile_v)


def topology_from_values(tr, classes, kind, thr, value_fn, active_fn=None, tile_fn=None):
    """Decided topology of the lower levels (Sec. 3.3, 3.5) from per-voxel functions.

    classes: level-1 class of every leaf slot of tr's level-1 nodes (0 = leaf).
    Inside every predicted leaf a voxel slot p is active where active_fn(p) holds
    (the level-0 classifier's decision); without one, where the value the
    regressor gives it passes the volume's own active rule: |v| <= band for a
    level set (closed interval, Sec. 3.2.1), v > threshold for fog.  value_fn(p)
    gives the values in value units; tile_fn as in topology_from_decisions.
    Returns leaf origins, voxel coordinates and values in canonical order, and the
    predicted tiles."""
    if active_fn is not None:
        def values(p, act):
            return value_fn(p[act])
        return topology_from_decisions(tr, classes, active_fn, values, tile_fn)
    cache = {}

    def active(p):
        v = np.asarray(value_fn(p), np.float64)
        cache["v"] = v
        return np.abs(v) <= thr if kind == T.SDF else v > thr

    def values(p, act):
        return cache["v"][act]
    return topology_from_decisions(tr, classes, active, values, tile_fn)


def decode_topology(tr, lo, D, kind, thr, value_scale, l1, reg, l0=None, fp8=False, tile=None):
    """Full decode with the networks: level-1 classes at every leaf slot, then the
    level-0 classifier (logit > 0) or, without one, the regressor's value tested
    with the volume's active rule (topology_from_values), then the regressor's
    values; with a tile value regressor, every slot classified as an active tile
    takes its value at the slot's leaf centre.  l1, reg, l0, tile: (theta, shapes, B)."""
    cls = l1_classes(decode_l1(*l1, tr, lo, D, fp8=fp8))
    tile_fn = None
    if tile is not None:
        def tile_fn(o):
            return _batched_predict(*tile, mlp.normalize_leaf_slot(o, lo, D), fp8=fp8)[:, 0] * value_scale

    def reg_values(p):
        return _batched_predict(*reg, mlp.normalize_voxel(p, lo, D), fp8=fp8)[:, 0] * value_scale

    active = None
    if l0 is not None:
        def active(p):
            return _batched_predict(*l0, mlp.normalize_voxel(p, lo, D), fp8=fp8)[:, 0] > 0
    return topology_from_values(tr, cls, kind, thr, reg_values, active, tile_fn)


def _voxel_keys(ijk):
    ijk = np.asarray(ijk, np.int64) + (1 << 20)
    return (ijk[:, 0] << 42) | (ijk[:, 1] << 21) | ijk[:, 2]


def errors_topology(true_ijk, true_values, pred_ijk, pred_values):
    """Voxel-level comparison: predicted voxels that are not active (fp), active
    voxels not predicted (fn), and max / RMS value error over the voxels in both."""
    kt, kp = _voxel_keys(true_ijk), _voxel_keys(pred_ijk)
    common, it, ip = np.intersect1d(kt, kp, assume_unique=True, return_indices=True)
    d = np.asarray(pred_values, np.float64)[ip] - np.asarray(true_values, np.float64)[it]
    return dict(n_true=len(kt), n_pred=len(kp), fp=len(kp) - len(common), fn=len(kt) - len(common),
                n_common=len(common), max_abs=float(np.max(np.abs(d))) if len(d) else 0.0,
                rms=float(np.sqrt(np.mean(d * d))) if len(d) else 0.0)


def errors(tr, vhat, kind, pred_mask=None):
    """Error report: max |v^ - v| and RMS over the true active voxels (value
    units), IoU of the interior {v <= 0} over the active set for level sets,
    and level-0 mask false positives / negatives when predicted masks are given."""
    v = tr["values"]
    d = np.asarray(vhat, np.float64) - v
    rep = dict(n=len(v), max_abs=float(np.max(np.abs(d))) if len(v) else 0.0,
               rms=float(np.sqrt(np.mean(d * d))) if len(v) else 0.0)
    if kind == T.SDF:
        a, b = v <= 0, np.asarray(vhat) <= 0
        union = int(np.sum(a | b))
        rep["iou"] = float(np.sum(a & b) / union) if union else 1.0
    if pred_mask is not None:
        truth = tr["leaf_mask"]
        fp = sum(bin(int(w)).count("1") for w in np.bitwise_and(pred_mask, ~truth).reshape(-1))
        fn = sum(bin(int(w)).count("1") for w in np.bitwise_and(~pred_mask, truth).reshape(-1))
        rep["fp"], rep["fn"] = int(fp), int(fn)
    return rep


def query_hits(tr, q):
    """Online random access, step 1 (Sec. 3.5): the explicit tree decides for each
    query position q (float, index space; voxel p covers [p, p+1) per axis) whether
    it falls on an active voxel.  The voxel is floor(q); it is a hit iff its leaf
    exists and the leaf's active mask holds it (the voxel is in the tree's active
    set).  Non-finite queries and queries outside int32 are misses."""
    q = np.asarray(q, np.float64).reshape(-1, 3)
    ok = np.all(np.isfinite(q), axis=1) & np.all(np.abs(q) < 2.0 ** 31 - 2, axis=1)
    p = np.zeros((len(q), 3), np.int64)
    p[ok] = np.floor(q[ok]).astype(np.int64)
    active = {tuple(v) for v in np.asarray(tr["ijk"], np.int64).tolist()}
    return np.array([bool(ok[i]) and tuple(p[i]) in active for i in range(len(q))], dtype=bool)


def query_tiles(tr, q):
    """Random access through the level-1 nodes (Sec. 3.3.1, 3.5): the active tile a
    query position falls in -- the tile whose leaf-sized region holds its voxel
    floor(q) -- as an index into the tree's tiles, or -1 (no level-1 node there, or
    the slot is a leaf or an inactive tile).  A voxel inside an existing leaf is
    never in a tile."""
    q = np.asarray(q, np.float64).reshape(-1, 3)
    ok = np.all(np.isfinite(q), axis=1) & np.all(np.abs(q) < 2.0 ** 31 - 2, axis=1)
    where = {tuple(o): t for t, o in enumerate(np.asarray(tr["tile_origin"], np.int64).tolist())}
    out = np.full(len(q), -1, np.int64)
    for i in np.nonzero(ok)[0]:
        o = tuple(int(c) & ~7 for c in np.floor(q[i]).astype(np.int64))
        out[i] = where.get(o, -1)
    return out


def query_values(theta, shapes, B, tr, lo, D, kind, band, q, background, tile=None):
    """Online random access of the [Hash,5,4,NN(3)] configuration (Sec. 3.5): a hit
    gets the regressor's value at its own position, normalised like the voxel
    centres, x = (q - lo) / D (so q = p + 1/2 reproduces the decode of voxel p),
    scaled back to value units; with a tile value regressor `tile` = (theta,
    shapes, B), a query in an active tile gets that regressor's value at the
    tile's leaf-slot centre (the tile's one value, as the tile decode gives it);
    every other query gets `background`.  Returns (values, hits) (hits: voxel hits)."""
    q = np.asarray(q, np.float64).reshape(-1, 3)
    hits = query_hits(tr, q)
    vals = np.full(len(q), float(background))
    if hits.any():
        x = (q[hits] - np.asarray(lo, np.float64)) / float(D)
        y = _batched_predict(theta, shapes, B, x)[:, 0]
        vals[hits] = y * band if kind == T.SDF else y
    if tile is not None:
        t = query_tiles(tr, q)
        sel = t >= 0
        if sel.any():
            vt = decode_tiles(*tile, tr, lo, D, kind, band)
            vals[sel] = vt[t[sel]]
    return vals, hits


def topology_patches(true_ijk, pred_ijk):
    """Patches (Sec. 3.3.1; Tab. memory_cost counts them at 12 bytes a coordinate):
    the predicted voxels that are not active (false positives) and the active
    voxels that were not predicted (false negatives), each list in the tree's
    canonical voxel order.  Removing the first list from the prediction and adding
    the second restores the true active set exactly."""
    kt, kp = _voxel_keys(true_ijk), _voxel_keys(pred_ijk)
    fp = np.asarray(pred_ijk, np.int64)[~np.isin(kp, kt)]
    fn = np.asarray(true_ijk, np.int64)[~np.isin(kt, kp)]

    def canonical(ijk):
        if len(ijk) == 0:
            return np.zeros((0, 3), np.int32)
        return T.build(ijk.astype(np.int32), np.zeros(len(ijk)))["ijk"]

    return canonical(fp), canonical(fn)
