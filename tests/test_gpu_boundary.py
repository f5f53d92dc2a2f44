"""GPU tests of the device-pointer boundary: the index-taking forward / backward
calls (samples gathered and normalised inside the kernels), their reserved
workspace and stream capture, the range check of sample indices, parameters
loaded from device memory and the autograd function training them, and a fit
across learning-rate decay steps against the oracle."""
import numpy as np
import pytest
import torch

import workloads
from oracle import fit as F, mlp, sampler as S, tree as T

pytestmark = pytest.mark.gpu
DEV = "cuda"

# (W, H, n_freq, n_out, net id, oracle network name)
NETS = [(64, 3, 18, 1, 0, "regressor"), (128, 3, 64, 1, 1, "l0"), (64, 4, 64, 3, 2, "l1")]


@pytest.fixture(scope="module")
def volume(gpu_lib):
    """A sphere on a box with a negative origin and a ragged extent (several level-1
    nodes and leaves at negative coordinates)."""
    v = workloads.sphere_sdf(n=80, center=(41.0, 38.0, 35.0), radius=30.0)[:, :77, :75].contiguous()
    origin = (-40, -9, 3)
    tr = gpu_lib.Tree(v.to(DEV), origin, T.SDF, 3.0)
    ot = T.build(*T.active_set_dense(v.numpy(), origin, T.SDF, 3.0))
    return tr, ot, origin


def make(gpu_lib, net, prec, lo, D, seed=3):
    W, H, m, c, k, _ = net
    B = workloads.pe_matrix(6) if m == 18 else workloads.ffm_matrix(m, 10.0, seed=seed + 1)
    th = workloads.init_params(2 * m, W, H, c, seed=seed)
    model = gpu_lib.Model({k: (W, H, m, c)}, precision=prec, domain_lo=lo, domain_size=D, value_scale=3.0)
    model.set_params(k, th)
    model.set_encoding(k, B)
    return model, th.astype(np.float64), B.astype(np.float64), mlp.layer_shapes(2 * m, W, H, c)


def kernel_coords(ot, name, idx, lo, D):
    """The normalised coordinates as the kernel forms them: float32 (p - lo + half) * (1 / D)."""
    idx = np.asarray(idx, np.int64)
    if name == "regressor":
        p, half = ot["ijk"][idx], 0.5
    elif name == "l0":
        p, half = ot["leaf_origin"][idx >> 9].astype(np.int64) + T.n0_to_offset(idx & 511), 0.5
    else:
        p, half = ot["l1_origin"][idx >> 12].astype(np.int64) + T.n1_to_offset(idx & 4095), 4.0
    inv = np.float32(1.0) / np.float32(D)
    return (((p - np.asarray(lo)).astype(np.float32) + np.float32(half)) * inv).astype(np.float32)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("net", NETS, ids=[n[5] for n in NETS])
def test_forward_dev_gathers_in_kernel(gpu_lib, volume, prec, net):
    """Outputs at population indices equal, bit for bit, the outputs at the coordinates
    the kernel forms from them, and match the oracle at the oracle's own coordinates."""
    tr, ot, origin = volume
    p = gpu_lib.FP32 if prec == "fp32" else gpu_lib.BF16
    lo, D = (origin[0] - 3, origin[1] + 2, origin[2] - 5), 90
    model, th, B, shapes = make(gpu_lib, net, p, lo, D)
    pop = F.population(ot, net[5])
    idx = np.random.default_rng(7).integers(0, pop, 5000)
    idx[:3] = [0, pop - 1, pop // 2]
    y = model.forward(net[4], tr, torch.from_numpy(idx.astype(np.int32)).to(DEV)).cpu().numpy()
    xk = kernel_coords(ot, net[5], idx, lo, D)
    yc = model.forward_coords(net[4], torch.from_numpy(xk).to(DEV)).cpu().numpy()
    assert np.array_equal(y, yc)
    x, _ = F.net_inputs(ot, net[5], idx, lo, D, T.SDF, 3.0)
    yo = mlp.predict(mlp.unflatten(th, shapes), x, B)
    err = np.max(np.abs(y - yo) / (1 + np.abs(yo)))
    assert err <= (1e-6 if p == gpu_lib.FP32 else 2e-3), err
    assert model.take_errors() == 0


@pytest.mark.parametrize("net", NETS, ids=[n[5] for n in NETS])
def test_backward_dev_matches_oracle(gpu_lib, volume, record, net):
    """FP32 gradient at population indices against the oracle, element-wise per tensor,
    on samples whose hidden pre-activations are all away from the ReLU kinks (bound
    1e-5: the first layer's gradient sums products with Fourier features of phases
    up to tens of revolutions, which carry the float32 phase's and the hardware
    sine's errors; measured 5e-6)."""
    tr, ot, origin = volume
    lo, D = (origin[0] - 3, origin[1] + 2, origin[2] - 5), 90
    model, th, B, shapes = make(gpu_lib, net, gpu_lib.FP32, lo, D)
    pop = F.population(ot, net[5])
    cand = np.random.default_rng(8).integers(0, pop, 6000)
    x, _ = F.net_inputs(ot, net[5], cand, lo, D, T.SDF, 3.0)
    _, cache = mlp.forward(mlp.unflatten(th, shapes), mlp.encode(x, B))
    zmin = np.min(np.stack([np.abs(cache[i]).min(axis=1) for i in range(1, len(cache), 2)]), axis=0)
    keep = zmin > 1e-5
    idx, x = cand[keep][:3000], x[keep][:3000]
    assert len(idx) == 3000
    gy = np.random.default_rng(9).standard_normal((len(idx), net[3]))
    model.reserve_dev(net[4], 4096)
    g = model.backward(net[4], tr, torch.from_numpy(idx.astype(np.int32)).to(DEV),
                       torch.from_numpy(gy.astype(np.float32)).to(DEV)).cpu().numpy().astype(np.float64)
    go = F.param_grad(th, shapes, B, x, gy.astype(np.float32).astype(np.float64))
    a, errs = 0, []
    for o, i in shapes:
        for n in (o * i, o):
            errs.append(np.max(np.abs(g[a:a + n] - go[a:a + n])) / np.max(np.abs(go[a:a + n])))
            a += n
    record("backward_dev_fp32_%s" % net[5], elem=max(errs))
    assert max(errs) <= 1e-5, errs


def test_dev_calls_need_reservation(gpu_lib, volume):
    tr, ot, origin = volume
    model, th, B, shapes = make(gpu_lib, NETS[0], gpu_lib.BF16, origin, 80)
    idx = torch.arange(100, dtype=torch.int32, device=DEV)
    gy = torch.ones(100, 1, device=DEV)
    with pytest.raises(gpu_lib.NvdbError) as e:
        model.backward(0, tr, idx, gy)
    assert e.value.code == gpu_lib.E_STATE
    model.reserve_dev(0, 64)
    with pytest.raises(gpu_lib.NvdbError) as e:
        model.backward(0, tr, idx, gy)
    assert e.value.code == gpu_lib.E_STATE
    with pytest.raises(gpu_lib.NvdbError) as e:
        model.reserve_dev(0, 0)
    assert e.value.code == gpu_lib.E_INVALID
    for bad in (idx.long(), idx.float(), idx.cpu(), torch.arange(200, dtype=torch.int32, device=DEV)[::2]):
        with pytest.raises(gpu_lib.NvdbError):
            model.forward(0, tr, bad)


def test_out_of_range_indices_are_counted(gpu_lib, volume):
    """An index at or beyond the population size is read as index 0 and counted; a
    fit with such an explicit order fails with E_INVALID."""
    tr, ot, origin = volume
    model, th, B, shapes = make(gpu_lib, NETS[0], gpu_lib.BF16, origin, 80)
    pop = len(ot["values"])
    idx = np.arange(1000, dtype=np.int64) % pop
    idx[[5, 17, 999]] = [pop, pop + 12345, 2 ** 32 - 1]
    t = torch.from_numpy(idx.astype(np.uint32).view(np.int32)).to(DEV)
    y = model.forward(0, tr, t).cpu().numpy()
    assert model.take_errors() == 3
    assert model.take_errors() == 0
    y0 = model.forward(0, tr, torch.zeros(1, dtype=torch.int32, device=DEV)).cpu().numpy()
    assert np.array_equal(y[[5, 17, 999]], np.repeat(y0, 3, axis=0))
    with pytest.raises(gpu_lib.NvdbError) as e:
        model.fit(tr, steps=2, batch=500, nets_mask=1, idx={0: t})
    assert e.value.code == gpu_lib.E_INVALID
    assert model.take_errors() == 0


def test_dev_calls_under_graph_capture(gpu_lib, volume):
    """forward_dev and backward_dev allocate nothing once reserved: recorded into a
    CUDA graph, every replay (with eager work between replays) equals the eager calls."""
    tr, ot, origin = volume
    model, th, B, shapes = make(gpu_lib, NETS[1], gpu_lib.BF16, origin, 80)
    pop = F.population(ot, "l0")
    n = 20000
    model.reserve_dev(1, n)
    idx = torch.from_numpy(np.random.default_rng(3).integers(0, pop, n).astype(np.int32)).to(DEV)
    gy = torch.randn(n, 1, device=DEV, generator=torch.Generator(DEV).manual_seed(5))
    y_ref = model.forward(1, tr, idx)
    g_ref = model.backward(1, tr, idx, gy)
    torch.cuda.synchronize()
    y_out = torch.empty_like(y_ref)
    g_out = torch.empty_like(g_ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        model.forward(1, tr, idx, out=y_out)  # warm-up outside the capture
        model.backward(1, tr, idx, gy, out=g_out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        model.forward(1, tr, idx, out=y_out)
        model.backward(1, tr, idx, gy, out=g_out)
    for r in range(3):
        y_out.zero_()
        g_out.fill_(float(r + 1))
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(y_out, y_ref), r
        assert torch.equal(g_out, g_ref), r
        _ = model.forward(1, tr, idx[: 1000 * (r + 1)])  # eager work between replays
        torch.cuda.synchronize()


def test_autograd_trains_parameter_tensor(gpu_lib, volume):
    """The autograd function reads the real parameter tensor: its gradient equals the
    backward call's, and torch's Adam on it lowers the regressor loss."""
    tr, ot, origin = volume
    model, th, B, shapes = make(gpu_lib, NETS[0], gpu_lib.BF16, origin, 80)
    pop = len(ot["values"])
    n = 1 << 14
    model.reserve_dev(0, n)
    vals = torch.from_numpy(ot["values"].astype(np.float32) / 3.0).to(DEV)
    Fn = gpu_lib.mlp_function()
    theta = torch.from_numpy(th.astype(np.float32)).to(DEV).requires_grad_(True)
    opt = torch.optim.Adam([theta], lr=3e-3)
    losses = []
    for step in range(30):
        idx = gpu_lib.sample_indices(0, 0, step, pop, n)
        y = Fn.apply(model, 0, tr, idx, theta)
        loss = ((y[:, 0] - vals[idx.long()]) ** 2).mean()
        opt.zero_grad()
        loss.backward()
        if step == 0:
            gy = (2.0 / n) * (y.detach()[:, 0] - vals[idx.long()])[:, None]
            assert torch.equal(theta.grad, model.backward(0, tr, idx, gy.contiguous()))
        opt.step()
        losses.append(float(loss))
    assert losses[-1] < 0.5 * losses[0], losses
    model.set_params_dev(0, theta.detach())
    assert torch.equal(model.get_params_dev(0), theta.detach())
    assert np.array_equal(model.get_params(0), theta.detach().cpu().numpy())


def test_fit_across_lr_decay_steps(gpu_lib, record):
    """FP32 fit of 10 steps with a staircase interval of 4 (the rate drops after steps 4
    and 8) against the oracle drawing the same samples: losses per step agree."""
    v = workloads.sphere_sdf()
    tr = gpu_lib.Tree(v.to(DEV), (0, 0, 0), T.SDF, 3.0)
    ot = T.build(*T.active_set_dense(v.numpy(), (0, 0, 0), T.SDF, 3.0))
    shapes = mlp.layer_shapes(36, 64, 3, 1)
    B = workloads.pe_matrix(6)
    th0 = workloads.init_params(36, 64, 3, 1, seed=4)
    model = gpu_lib.Model({0: (64, 3, 18, 1)}, precision=gpu_lib.FP32, domain_size=64, value_scale=3.0)
    model.set_params(0, th0)
    model.set_encoding(0, B)
    lr, decay, interval = 3e-3, 0.3, 4
    losses = model.fit(tr, steps=10, batch=4096, nets_mask=1, seed=9, lr=lr, lr_decay=decay, lr_interval=interval)[0]
    tho, _, _, lo = F.train(th0.astype(np.float64), shapes, B.astype(np.float64), ot, "regressor", (0, 0, 0), 64,
                            T.SDF, 3.0, steps=10, batch=4096, seed=9, lr0=lr, decay=decay, interval=interval)
    assert [mlp.lr_at(s, lr, decay, interval) for s in (1, 4, 5, 8, 9)] == [lr, lr, lr * decay, lr * decay,
                                                                           lr * decay ** 2]
    rel = np.abs(losses - lo) / np.abs(lo)
    record("fit_lr_decay_fp32", loss_rel=rel.max())
    assert rel.max() <= 1e-5, rel
    thg = model.get_params(0).astype(np.float64)
    assert np.linalg.norm(thg - tho) / np.linalg.norm(tho - th0) <= 2e-2
    # the same schedule with no decay takes other steps: the decay is exercised
    th_nd, _, _, lo_nd = F.train(th0.astype(np.float64), shapes, B.astype(np.float64), ot, "regressor", (0, 0, 0),
                                 64, T.SDF, 3.0, steps=10, batch=4096, seed=9, lr0=lr, decay=1.0, interval=interval)
    assert np.abs(lo_nd[-1] - lo[-1]) / lo[-1] > 1e-3


@pytest.mark.parametrize("net", [(128, 4, 64, 1, 0, "regressor"), (128, 3, 64, 1, 1, "l0")], ids=["4x128", "3x128"])
def test_classic_train_kernel_128_bf16(gpu_lib, volume, record, net, monkeypatch):
    """The 128-wide BF16 networks train with the activation-rows kernel; the classic
    kernel (activations in registers, layer 1's gradient in LDS), still used for the
    other shapes, is selected for them by NVDB_TRAIN_CLASSIC at model creation.  Both
    give the oracle's BF16-form gradient on the same samples."""
    from oracle import bf16 as bf16_form
    tr, ot, origin = volume
    lo, D = (origin[0] - 3, origin[1] + 2, origin[2] - 5), 90
    pop = F.population(ot, net[5])
    idx = np.random.default_rng(12).integers(0, pop, 3000)
    gy = np.random.default_rng(13).standard_normal((len(idx), 1)).astype(np.float32)
    x, _ = F.net_inputs(ot, net[5], idx, lo, D, T.SDF, 3.0)
    grads = {}
    for kernel in ("rows", "classic"):
        if kernel == "classic":
            monkeypatch.setenv("NVDB_TRAIN_CLASSIC", "1")
        model, th, B, shapes = make(gpu_lib, net, gpu_lib.BF16, lo, D)
        monkeypatch.delenv("NVDB_TRAIN_CLASSIC", raising=False)
        model.reserve_dev(net[4], len(idx))
        grads[kernel] = model.backward(net[4], tr, torch.from_numpy(idx.astype(np.int32)).to(DEV),
                                       torch.from_numpy(gy).to(DEV)).cpu().numpy().astype(np.float64)
    params = mlp.unflatten(th, shapes)
    _, cb = bf16_form.forward_bf16(params, mlp.encode(x, B))
    gb = mlp.flatten(bf16_form.backward_bf16(params, cb, gy.astype(np.float64)))
    for kernel, g in grads.items():
        a, errs = 0, []
        for o, i in shapes:
            for n in (o * i, o):
                errs.append(np.max(np.abs(g[a:a + n] - gb[a:a + n])) / np.max(np.abs(gb[a:a + n])))
                a += n
        record("classic_vs_rows_%s_%s" % (net[5], kernel), elem_bf16_form=max(errs))
        assert max(errs) <= 0.1, (kernel, errs)
