"""The 1024^3 fog volume at full size (fBm cloud, 6 octaves, active where the
density exceeds 0.55; 2.7e8 voxels, 6.4e5 leaves, 469 level-1 nodes), in the
launch configuration the benchmark times: the tree against the oracle's build of
whole sampled leaves and level-1 nodes plus full-size counts; the BF16 and FP8
regressor decode on the voxels of sampled leaves; level-1 classes on sampled
nodes; the decode of the whole lower tree restricted to sampled level-1 nodes,
voxel by voxel.  The oracle evaluates the library's fitted weights."""
import numpy as np
import pytest
import torch

import workloads
from oracle import bf16 as bf16_form, fit as F, mlp, tree as T

pytestmark = pytest.mark.gpu
DEV = "cuda"
THR = 0.55
N_GRID = 1024
M, W, H = 64, 128, 4
BF16_FWD_TOL = 2e-3        # BF16 decode against the FP64 oracle, |dy| / (1 + |y|)
BF16_FORM_FWD_TOL = 1e-3   # against the oracle's BF16 form
FP8_TOL = 3e-2             # FP8 decode against the FP8 oracle
REG = (W, H, M, 1)
L1 = (64, 4, M, 3)


def _keys(ijk):
    return F._voxel_keys(np.asarray(ijk, np.int64))


@pytest.fixture(scope="module")
def c3(gpu_lib):
    g = workloads.fbm_cloud(N_GRID, device=DEV)
    tr = gpu_lib.Tree(g, (0, 0, 0), T.FOG, THR)
    return g, tr, tr.export()


def mini_tree(g, origins, n):
    """Oracle tree of the voxels inside the blocks of edge n at `origins` (whole
    leaves for n = 8, whole level-1 nodes for n = 128)."""
    ijk, vals = [], []
    for o in np.asarray(origins).reshape(-1, 3):
        x, y, z = (int(c) for c in o)
        blk = g[x:x + n, y:y + n, z:z + n].cpu().numpy()
        a, v = T.active_set_dense(blk, (x, y, z), T.FOG, THR)
        ijk.append(a)
        vals.append(v)
    return T.build(np.concatenate(ijk), np.concatenate(vals))


def test_c3_tree_full_size(gpu_lib, c3):
    g, tr, ex = c3
    info = tr.info()
    act = g > THR
    assert info.n_voxels == int(act.sum())
    # leaves and level-1 nodes: exactly the 8^3 / 128^3 blocks holding an active voxel
    lb = act.view(128, 8, 128, 8, 128, 8).any(dim=5).any(dim=3).any(dim=1)
    want = torch.nonzero(lb).cpu().numpy() * 8
    assert info.n_leaves == len(want) == len(ex["leaf_origin"])
    assert np.array_equal(np.sort(_keys(ex["leaf_origin"])), np.sort(_keys(want)))
    nb = lb.view(8, 16, 8, 16, 8, 16).any(dim=5).any(dim=3).any(dim=1)
    want1 = torch.nonzero(nb).cpu().numpy() * 128
    assert info.n_l1 == len(want1) == len(ex["l1_origin"])
    assert np.array_equal(np.sort(_keys(ex["l1_origin"])), np.sort(_keys(want1)))
    del act, lb, nb
    assert int(ex["leaf_off"][-1]) == info.n_voxels
    rng = np.random.default_rng(0)
    # 64 sampled leaves: origin, mask, offset span and values bit-exact
    leaves = np.sort(rng.choice(info.n_leaves, 64, replace=False))
    mt = mini_tree(g, ex["leaf_origin"][leaves], 8)
    assert np.array_equal(mt["leaf_origin"], ex["leaf_origin"][leaves])
    assert np.array_equal(mt["leaf_mask"], ex["leaf_mask"][leaves])
    for j, li in enumerate(leaves):
        a, b = int(ex["leaf_off"][li]), int(ex["leaf_off"][li + 1])
        assert b - a == mt["leaf_off"][j + 1] - mt["leaf_off"][j]
        assert np.array_equal(ex["values"][a:b].astype(np.float64), mt["values"][mt["leaf_off"][j]:mt["leaf_off"][j + 1]])
    # 3 sampled level-1 nodes, whole: child masks, their leaves (contiguous in canonical order), values
    for node in rng.choice(info.n_l1, 3, replace=False):
        o = ex["l1_origin"][node]
        mn = mini_tree(g, o, 128)
        assert np.array_equal(mn["l1_origin"][0], o) and np.array_equal(mn["l1_child"][0], ex["l1_child"][node])
        inn = np.nonzero(np.all((ex["leaf_origin"] & ~127) == o, axis=1))[0]
        assert len(inn) == len(mn["leaf_origin"]) and np.all(np.diff(inn) == 1)
        assert np.array_equal(ex["leaf_origin"][inn], mn["leaf_origin"])
        assert np.array_equal(ex["leaf_mask"][inn], mn["leaf_mask"])
        a, b = int(ex["leaf_off"][inn[0]]), int(ex["leaf_off"][inn[-1] + 1])
        assert np.array_equal(ex["values"][a:b].astype(np.float64), mn["values"])


@pytest.fixture(scope="module")
def c3_model(gpu_lib, c3):
    """The benchmark's cloud networks (BF16 regressor 4x128 and level-1 classifier
    4x64, Fourier features m = 64, sigma 10), fitted for 300 steps of 2^18 samples
    per network at 128 work-groups per network."""
    _, tr, _ = c3
    m = gpu_lib.Model({0: REG, 2: L1}, precision=gpu_lib.BF16, domain_size=N_GRID, value_scale=1.0)
    Bs = {0: workloads.ffm_matrix(M, 10.0, seed=51), 2: workloads.ffm_matrix(M, 10.0, seed=52)}
    for k, (w, h, mm, c) in ((0, REG), (2, L1)):
        m.set_encoding(k, Bs[k])
        m.set_params(k, workloads.init_params(2 * mm, w, h, c, seed=53 + k))
    m.set_train_groups(128)
    m.fit(tr, steps=300, batch=1 << 18, nets_mask=0b101, seed=0, lr=1e-3)

    def net(k, shape):
        w, h, mm, c = shape
        return m.get_params(k).astype(np.float64), mlp.layer_shapes(2 * mm, w, h, c), Bs[k].astype(np.float64)
    return m, net(0, REG), net(2, L1)


def test_c3_decode_sampled(gpu_lib, c3, c3_model):
    g, tr, ex = c3
    m, reg, l1 = c3_model
    values, _ = m.decode(tr, values=True, masks=False)
    v8, _ = m.decode(tr, values=True, masks=False, fp8=True)
    rng = np.random.default_rng(5)
    leaves = np.sort(rng.choice(len(ex["leaf_origin"]), 16, replace=False))
    mt = mini_tree(g, ex["leaf_origin"][leaves], 8)
    sel = np.concatenate([np.arange(ex["leaf_off"][li], ex["leaf_off"][li + 1]) for li in leaves])
    assert len(sel) == len(mt["values"]) >= 1000
    vg = values.cpu().numpy()[sel].astype(np.float64)
    vo = F.decode_values(*reg, mt, (0, 0, 0), N_GRID, T.FOG, 1.0)
    assert np.max(np.abs(vg - vo) / (1 + np.abs(vo))) <= BF16_FWD_TOL
    x = mlp.normalize_voxel(mt["ijk"], (0, 0, 0), N_GRID)
    yb, _ = bf16_form.forward_bf16(mlp.unflatten(reg[0], reg[1]), mlp.encode(x, reg[2]))
    assert np.max(np.abs(vg - yb[:, 0]) / (1 + np.abs(yb[:, 0]))) <= BF16_FORM_FWD_TOL
    vo8 = F.decode_values(*reg, mt, (0, 0, 0), N_GRID, T.FOG, 1.0, fp8=True)
    assert np.max(np.abs(v8.cpu().numpy()[sel] - vo8)) <= FP8_TOL
    # level-1 classes of every leaf slot of 4 sampled nodes (BF16 and FP8), away from ties
    cls = m.decode_l1(tr).cpu().numpy()
    cls8 = m.decode_l1(tr, fp8=True).cpu().numpy()
    nodes = np.sort(rng.choice(len(ex["l1_origin"]), 4, replace=False))
    sub = {"l1_origin": ex["l1_origin"][nodes], "l1_child": ex["l1_child"][nodes],
           "l1_active": np.zeros((len(nodes), 64), np.uint64)}
    for got, f8, margin in ((cls, False, 2 * BF16_FWD_TOL * 8), (cls8, True, 2 * FP8_TOL)):
        lg = F.decode_l1(*l1, sub, (0, 0, 0), N_GRID, fp8=f8)
        srt = np.sort(lg, axis=1)
        tie = (srt[:, -1] - srt[:, -2]) <= margin
        ok = (got[nodes].reshape(-1) == F.l1_classes(lg)) | tie
        assert ok.all(), (f8, int((~ok).sum()))


def test_c3_topology_decode_sampled(gpu_lib, c3, c3_model):
    """The decode of the lower levels (level-1 classes -> leaves -> the regressor
    tested with the fog rule -> values) against the oracle on two sampled level-1
    nodes: leaves differ only at near-tie slots, voxels of leaves both sides
    predict differ only where the oracle's value lies within BF16 rounding of the
    threshold, values of common voxels within the BF16 bound."""
    g, tr, ex = c3
    m, reg, l1 = c3_model
    pred = m.decode_topology(tr)
    pe = pred.export()
    rng = np.random.default_rng(9)
    node_of = pe["leaf_origin"] & ~127
    uk, cnt = np.unique(_keys(node_of), return_counts=True)
    count = dict(zip(uk.tolist(), cnt.tolist()))
    per_node = np.array([count.get(k, 0) for k in _keys(ex["l1_origin"]).tolist()])
    # the quarter of the nodes with the fewest predicted leaves (at least 20): the
    # oracle evaluates the regressor at every voxel slot of a node's leaves
    order = [n for n in np.argsort(per_node, kind="stable") if per_node[n] >= 20]
    cand = order[:max(2, len(order) // 4)]
    assert len(cand) >= 2
    vtol = lambda v: BF16_FWD_TOL * (1 + np.abs(v))
    for node in rng.choice(cand, 2, replace=False):
        o = ex["l1_origin"][node]
        sub = {"l1_origin": o[None], "l1_child": ex["l1_child"][node][None], "l1_active": np.zeros((1, 64), np.uint64)}
        lg = F.decode_l1(*l1, sub, (0, 0, 0), N_GRID)
        srt = np.sort(lg, axis=1)
        tie = (srt[:, -1] - srt[:, -2]) <= 2 * BF16_FWD_TOL * 8
        cache = {}

        def value_fn(p):
            v = F._batched_predict(*reg, mlp.normalize_voxel(p, (0, 0, 0), N_GRID))[:, 0]
            cache["p"], cache["v"] = p, v
            return v
        od = F.topology_from_values(sub, F.l1_classes(lg), T.FOG, THR, value_fn)
        # leaves
        inn = np.nonzero(np.all(node_of == o, axis=1))[0]
        kg, ko = _keys(pe["leaf_origin"][inn]), _keys(od["leaf_origin"])
        slot_keys = _keys(o[None, :].astype(np.int64) + T.n1_to_offset(np.arange(4096)))
        assert np.isin(np.setxor1d(kg, ko), slot_keys[tie]).all()
        # voxels of the leaves both sides predict, slot by slot
        both = np.intersect1d(kg, ko)
        gi = inn[np.isin(kg, both)]
        slots_g = (pe["leaf_origin"][gi][:, None, :].astype(np.int64) + T.n0_to_offset(np.arange(512))[None]).reshape(-1, 3)
        bits = np.unpackbits(pe["leaf_mask"][gi].view(np.uint8), bitorder="little").astype(bool)
        ok_p = np.isin(_keys(cache["p"]), _keys(slots_g))
        vo_slot = dict(zip(_keys(cache["p"][ok_p]).tolist(), cache["v"][ok_p].tolist()))
        vs = np.array([vo_slot[k] for k in _keys(slots_g).tolist()])
        act_o = vs > THR
        flip = bits != act_o
        assert np.all(np.abs(vs[flip] - THR) <= vtol(vs[flip])), int(flip.sum())
        # values where both sides mark the voxel
        a = pe["leaf_off"]
        gv = np.concatenate([pe["values"][a[i]:a[i + 1]] for i in gi]).astype(np.float64)
        common = bits & act_o
        assert len(gv) == int(bits.sum())
        assert np.all(np.abs(gv[common[bits]] - vs[common]) <= vtol(vs[common]))
