"""nvdb_query_noalloc (random access with its scratch in a static per-GPU device
array, no allocation inside the call) against nvdb_query on the same inputs:
two calls in a row, the second with a smaller input, each equal to the
allocating call (hit flags bit for bit, values bit for bit: the same kernels
evaluate each hit independently of where the compaction put it), on a level
set and on a fog whose active tiles (Sec. 3.3.1) the tile regressor serves."""
import numpy as np
import pytest
import torch

import workloads
from oracle import tree as T

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_query_noalloc_matches_query(gpu_lib):
    v = workloads.sphere_sdf(n=96, center=(47.0, 50.0, 44.0), radius=35.0)
    tr = gpu_lib.Tree(v.to(DEV), (-20, 5, 0), T.SDF, 3.0)
    K, W, H, m = 128, 128, 4, 64
    model = gpu_lib.Model({0: (W, H, m, 1)}, precision=gpu_lib.BF16, domain_lo=(-20, 5, 0), domain_size=96,
                          value_scale=3.0)
    model.set_params(0, workloads.init_params(K, W, H, 1, seed=2))
    model.set_encoding(0, workloads.ffm_matrix(m, 10.0, seed=3))
    rng = np.random.default_rng(11)
    # first call: 150,000 positions (three batches of 65,536, the last ragged), about a
    # third of them at active voxels; second call: 1,000 positions in one batch
    ex = tr.export()
    mask_bits = np.unpackbits(ex["leaf_mask"].view(np.uint8), bitorder="little").reshape(-1, 512)
    leaf, n0 = np.nonzero(mask_bits)
    act = ex["leaf_origin"][leaf] + np.stack([n0 >> 6, (n0 >> 3) & 7, n0 & 7], 1)
    for n, batch in ((150_000, 0), (1_000, 4096)):
        q = rng.uniform(-25, 120, (n, 3))
        on = rng.random(n) < 0.35
        q[on] = act[rng.integers(0, len(act), on.sum())] + rng.random((on.sum(), 3))
        q[::997] = np.nan
        qd = torch.from_numpy(q.astype(np.float32)).to(DEV)
        v_ref, h_ref = model.query(tr, qd, background=7.5, batch=batch, return_hits=True)
        hits = torch.full((n,), 9, dtype=torch.uint8, device=DEV)
        vals = torch.full((n,), -1.0, device=DEV)
        model.query_noalloc(tr, qd, background=7.5, batch=batch, values=vals, hits=hits)
        torch.cuda.synchronize()
        assert torch.equal(hits, h_ref)
        assert 0.2 < float(h_ref.float().mean()) < 0.5
        assert torch.equal(vals, v_ref)
    with pytest.raises(gpu_lib.NvdbError) as e:
        model.query_noalloc(tr, qd, background=7.5, batch=65537, values=vals, hits=hits)
    assert e.value.code == gpu_lib.E_INVALID


def test_query_noalloc_with_tiles_matches_query(gpu_lib):
    v = workloads.saturated_fog(n=128, center=(64.0, 67.0, 62.0), radius=56.32, scale=32.0)
    tr = gpu_lib.Tree(v.to(DEV), (0, 0, 0), T.FOG, 0.05).prune_tiles()
    ot = T.prune_tiles(T.build(*T.active_set_dense(v.numpy(), (0, 0, 0), T.FOG, 0.05)))
    assert tr.info().n_tiles == len(ot["tile_value"]) >= 100
    nets = {0: (128, 4, 64, 1), 3: (64, 3, 18, 1)}
    model = gpu_lib.Model(nets, precision=gpu_lib.BF16, domain_size=128, value_scale=1.0)
    model.set_params(0, workloads.init_params(128, 128, 4, 1, seed=4))
    model.set_encoding(0, workloads.ffm_matrix(64, 10.0, seed=5))
    model.set_params(3, workloads.init_params(36, 64, 3, 1, seed=6))
    model.set_encoding(3, workloads.pe_matrix(6))
    rng = np.random.default_rng(12)
    # first call: 150,000 positions (three batches, the last ragged), a quarter in
    # active tiles and a quarter at active voxels; second call: 1,000 in one batch
    for n, batch in ((150_000, 0), (1_000, 4096)):
        q = rng.uniform(-10, 140, (n, 3))
        kind = rng.integers(0, 4, n)
        it, iv = kind == 0, kind == 1
        q[it] = ot["tile_origin"][rng.integers(0, len(ot["tile_origin"]), it.sum())] + rng.uniform(0, 8, (it.sum(), 3))
        q[iv] = ot["ijk"][rng.integers(0, len(ot["ijk"]), iv.sum())] + rng.random((iv.sum(), 3))
        q[::991] = np.nan
        qd = torch.from_numpy(q.astype(np.float32)).to(DEV)
        v_ref, h_ref = model.query(tr, qd, background=-2.0, batch=batch, return_hits=True)
        hits = torch.full((n,), 9, dtype=torch.uint8, device=DEV)
        vals = torch.full((n,), -1.0, device=DEV)
        model.query_noalloc(tr, qd, background=-2.0, batch=batch, values=vals, hits=hits)
        torch.cuda.synchronize()
        assert torch.equal(hits, h_ref)
        assert float((h_ref == 2).float().mean()) > 0.2 and float((h_ref == 1).float().mean()) > 0.2
        assert torch.equal(vals, v_ref)
