"""Compact serialised NeuralVDB (the upper levels explicit, the lower levels as
16-bit networks, Sec. 3.3.2 and Sec. 4; 12-byte patch coordinates, Tab.
memory_cost): the byte image read back by a parser written here from the
documented layout, the 16-bit codes equal to numpy's and torch's round to
nearest even, the patches equal to the difference between the truth and the
topology the 16-bit networks decode, the decoded volume's topology equal to
the truth, its values equal to the regressor with the stored weights, and
corrupt images rejected."""
import struct

import numpy as np
import pytest
import torch

import workloads
from oracle import tree as T

pytestmark = pytest.mark.gpu
DEV = "cuda"

HEADER = struct.Struct("<4sIIIiiff3ii3i3iII5q")
assert HEADER.size == 120


def parse(buf, param_count):
    """Sections of an archive image; param_count(W, H, n_freq, C) gives P."""
    f = HEADER.unpack_from(buf, 0)
    hd = dict(magic=f[0], version=f[1], flags=f[2], storage=f[3], precision=f[4], rule_kind=f[5], rule_thr=f[6],
              value_scale=f[7], domain_lo=f[8:11], domain_size=f[11], grid_origin=f[12:15], grid_dims=f[15:18],
              nets_mask=f[18], n_l2=f[20], n_l1=f[21], n_fp=f[22], n_fn=f[23], n_leaf=f[24])
    pos = HEADER.size
    l2o, l2c = [], []
    for _ in range(hd["n_l2"]):
        l2o.append(np.frombuffer(buf, np.int32, 3, pos))
        l2c.append(np.frombuffer(buf, np.uint64, 512, pos + 12))
        pos += 12 + 4096
    l1o, l1c, l1a = [], [], []
    explicit = bool(hd["flags"] & 1)
    for _ in range(hd["n_l1"]):
        l1o.append(np.frombuffer(buf, np.int32, 3, pos))
        pos += 12
        if explicit:
            l1c.append(np.frombuffer(buf, np.uint64, 64, pos))
            l1a.append(np.frombuffer(buf, np.uint64, 64, pos + 512))
            pos += 1024
    leaf_mask = np.frombuffer(buf, np.uint64, 8 * hd["n_leaf"], pos).reshape(-1, 8)
    pos += 64 * hd["n_leaf"]
    nets = {}
    for k in range(3):
        if not (hd["nets_mask"] >> k) & 1:
            continue
        W, H, nf, C = np.frombuffer(buf, np.int32, 4, pos).tolist()
        sin_freq = float(np.frombuffer(buf, np.float32, 1, pos + 16)[0])
        pos += 20
        B = np.frombuffer(buf, np.float32, 3 * nf, pos).reshape(nf, 3)
        pos += 12 * nf
        P = param_count(W, H, nf, C)
        codes = np.frombuffer(buf, np.uint16, P, pos)
        pos += (2 * P + 3) & ~3
        nets[k] = dict(shape=(W, H, nf, C), sin_freq=sin_freq, B=B, codes=codes)
    fp = np.frombuffer(buf, np.int32, 3 * hd["n_fp"], pos).reshape(-1, 3)
    pos += 12 * hd["n_fp"]
    fn = np.frombuffer(buf, np.int32, 3 * hd["n_fn"], pos).reshape(-1, 3)
    pos += 12 * hd["n_fn"]
    return dict(header=hd, l2_origin=np.array(l2o).reshape(-1, 3), l2_child=np.array(l2c).reshape(-1, 512),
                l1_origin=np.array(l1o).reshape(-1, 3), l1_child=np.array(l1c).reshape(-1, 64),
                l1_active=np.array(l1a).reshape(-1, 64), leaf_mask=leaf_mask, nets=nets, fp=fp, fn=fn, end=pos)


def n_params(W, H, nf, C):
    K = 2 * nf
    return K * W + W + (H - 1) * (W * W + W) + W * C + C


def archive_size(n_l2, n_l1, explicit_l1, n_leaf, shapes, n_fp, n_fn):
    """Bytes of the image by the documented layout (n_leaf: leaf masks stored)."""
    nets = sum(20 + 12 * nf + ((2 * n_params(W, H, nf, C) + 3) & ~3) for W, H, nf, C in shapes)
    return (120 + n_l2 * (12 + 4096) + n_l1 * (12 + (1024 if explicit_l1 else 0)) + 64 * n_leaf + nets
            + 12 * (n_fp + n_fn))


def codes16(theta, storage, lib):
    if storage == lib.STORE_F16:
        return theta.astype(np.float16).view(np.uint16)
    return torch.from_numpy(theta).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)


NETS = {0: (64, 3, 18, 1), 1: (64, 3, 18, 1), 2: (64, 4, 64, 3)}
ENC = {0: lambda: workloads.pe_matrix(6), 1: lambda: workloads.pe_matrix(6),
       2: lambda: workloads.ffm_matrix(64, 3.0, seed=4)}


@pytest.fixture(scope="module")
def fitted(gpu_lib):
    """A level set with a trained regressor, level-0 and level-1 classifiers (FP32 and BF16)."""
    v = workloads.sphere_sdf(n=200, center=(100.0, 90.0, 110.0), radius=70.0)
    tr = gpu_lib.Tree(v.to(DEV), (0, 0, 0), T.SDF, 3.0)
    out = {"tree": tr}
    for name, prec in (("fp32", gpu_lib.FP32), ("bf16", gpu_lib.BF16)):
        m = gpu_lib.Model(NETS, precision=prec, domain_size=256, value_scale=3.0)
        for k, (W, H, nf, C) in NETS.items():
            m.set_params(k, workloads.init_params(2 * nf, W, H, C, seed=40 + k))
            m.set_encoding(k, ENC[k]())
        m.fit(tr, steps=150, batch=4096, nets_mask=7, seed=1, lr=3e-3)
        out[name] = m
    return out


def rounded(gpu_lib, m, prec, mask, storage):
    """The model the archive holds: the networks of `mask` with 16-bit weights."""
    r = gpu_lib.Model({k: NETS[k] for k in NETS if (mask >> k) & 1}, precision=prec, domain_size=256,
                      value_scale=3.0)
    for k in NETS:
        if (mask >> k) & 1:
            r.set_params16(k, storage, m.get_params16(k, storage))
            r.set_encoding(k, ENC[k]())
    return r


CASES = [  # (precision, storage, networks, level-1 masks stored, leaf masks stored)
    ("fp32", "f16", 0b111, False, False),
    ("bf16", "bf16", 0b101, False, False),
    ("bf16", "f16", 0b011, True, False),
    ("fp32", "bf16", 0b001, True, False),
    ("bf16", "f16", 0b001, True, True),
]


@pytest.mark.parametrize("prec,store,mask,explicit,explicit_l0", CASES)
def test_archive_round_trip(gpu_lib, fitted, prec, store, mask, explicit, explicit_l0):
    tr = fitted["tree"]
    m = fitted[prec]
    P = gpu_lib.FP32 if prec == "fp32" else gpu_lib.BF16
    S = gpu_lib.STORE_F16 if store == "f16" else gpu_lib.STORE_BF16
    patches = not explicit_l0
    buf = gpu_lib.archive_write(m, tr, mask, S, explicit_l1=explicit, patches=patches, explicit_l0=explicit_l0)
    a = parse(buf, n_params)
    hd = a["header"]
    flags = (1 if explicit else 0) | (2 if patches else 0) | (4 if explicit_l0 else 0)
    assert hd["magic"] == b"NVDB" and hd["version"] == 1 and hd["flags"] == flags
    assert (hd["storage"], hd["precision"], hd["rule_kind"], hd["nets_mask"]) == (S, P, T.SDF, mask)
    assert hd["rule_thr"] == 3.0 and hd["value_scale"] == 3.0 and hd["domain_size"] == 256
    assert hd["domain_lo"] == (0, 0, 0)
    ti, ex = tr.info(), tr.export()
    assert hd["grid_origin"] == tuple(ti.grid_origin) and hd["grid_dims"] == tuple(ti.grid_dims)
    # sizes: the parser ends where the image ends, and the layout's accounting agrees
    shapes = [NETS[k] for k in range(3) if (mask >> k) & 1]
    assert hd["n_leaf"] == (ti.n_leaves if explicit_l0 else 0)
    assert a["end"] == len(buf) == archive_size(ti.n_l2, ti.n_l1, explicit, hd["n_leaf"], shapes, hd["n_fp"],
                                                hd["n_fn"])
    # upper levels as the tree holds them
    l2o, l2c = tr.export_l2()
    assert np.array_equal(a["l2_origin"], l2o) and np.array_equal(a["l2_child"], l2c)
    assert np.array_equal(a["l1_origin"], ex["l1_origin"])
    if explicit:
        assert np.array_equal(a["l1_child"], ex["l1_child"]) and not a["l1_active"].any()
    if explicit_l0:
        assert np.array_equal(a["leaf_mask"], ex["leaf_mask"])
    # networks: shapes, encodings exactly, parameters as round-to-nearest-even 16-bit codes
    for k, net in a["nets"].items():
        assert net["shape"] == NETS[k] and net["sin_freq"] == 0.0
        assert np.array_equal(net["B"], ENC[k]().astype(np.float32))
        assert np.array_equal(net["codes"], codes16(m.get_params(k), S, gpu_lib))
    # patches: the difference between the truth and what the stored networks decode
    r = rounded(gpu_lib, m, P, mask, S)
    pred = r.decode_topology(tr)
    if patches:
        fp, fn = gpu_lib.topology_patches(tr, pred)
        assert np.array_equal(a["fp"], fp.cpu().numpy()) and np.array_equal(a["fn"], fn.cpu().numpy())
    else:
        assert hd["n_fp"] == 0 and hd["n_fn"] == 0
    # decode: the true topology exactly, the values of the stored regressor
    dt, info = gpu_lib.archive_decode(buf)
    assert (info.n_l2, info.n_l1, info.n_fp, info.n_fn) == (ti.n_l2, ti.n_l1, hd["n_fp"], hd["n_fn"])
    de = dt.export()
    for key in ("leaf_origin", "leaf_mask", "leaf_off", "l1_origin"):
        assert np.array_equal(de[key], ex[key]), key
    want, _ = r.decode(tr, values=True, masks=False)
    assert np.array_equal(de["values"], want.cpu().numpy())
    if explicit_l0:
        return
    # without patches the image decodes to what the networks predict, no more
    buf0 = gpu_lib.archive_write(m, tr, mask, S, explicit_l1=explicit, patches=False)
    assert len(buf0) == len(buf) - 12 * (hd["n_fp"] + hd["n_fn"])
    d0, i0 = gpu_lib.archive_decode(buf0)
    pe, e0 = pred.export(), d0.export()
    assert i0.n_fp == 0 and i0.n_fn == 0
    for key in ("leaf_origin", "leaf_mask", "leaf_off", "values"):
        assert np.array_equal(e0[key], pe[key]), key


def test_archive_patches_are_used(gpu_lib, fitted):
    """The fitted networks leave patches to apply (else the round trip shows nothing)."""
    tr = fitted["tree"]
    buf = gpu_lib.archive_write(fitted["fp32"], tr, 0b001, gpu_lib.STORE_F16, explicit_l1=True)
    hd = parse(buf, n_params)["header"]
    assert hd["n_fp"] + hd["n_fn"] > 0


def test_archive_rejects_corrupt_images(gpu_lib, fitted):
    tr = fitted["tree"]
    buf = gpu_lib.archive_write(fitted["bf16"], tr, 0b101, gpu_lib.STORE_BF16)
    a = parse(buf, n_params)
    bad = [buf[:-1], buf + b"\0\0\0\0", b"NVDX" + buf[4:], buf[:4] + struct.pack("<I", 2) + buf[8:], b"",
           buf[:HEADER.size]]
    off = a["end"] - 12 * (a["header"]["n_fp"] + a["header"]["n_fn"])
    if a["header"]["n_fp"] > 0:  # a false-positive patch naming a voxel the decoded tree lacks
        bad.append(buf[:off] + struct.pack("<3i", -4096, -4096, -4096) + buf[off + 12:])
    if a["header"]["n_fp"] > 1:  # the same voxel removed twice
        bad.append(buf[:off + 12] + buf[off:off + 12] + buf[off + 24:])
    # an unaligned level-1 origin
    l1 = HEADER.size + a["header"]["n_l2"] * (12 + 4096)
    bad.append(buf[:l1] + struct.pack("<i", 5) + buf[l1 + 4:])
    for i, b in enumerate(bad):
        with pytest.raises(gpu_lib.NvdbError) as e:
            gpu_lib.archive_decode(b)
        assert e.value.code == gpu_lib.E_INVALID, i
    # stored leaf masks whose count disagrees with the header
    b5 = gpu_lib.archive_write(fitted["bf16"], tr, 0b001, gpu_lib.STORE_F16, explicit_l1=True, explicit_l0=True)
    n_leaf_at = HEADER.size - 8
    n_leaf = struct.unpack_from("<q", b5, n_leaf_at)[0]
    assert n_leaf == tr.info().n_leaves
    for wrong in (n_leaf - 1, n_leaf + 1, -1):
        with pytest.raises(gpu_lib.NvdbError) as e:
            gpu_lib.archive_decode(b5[:n_leaf_at] + struct.pack("<q", wrong) + b5[HEADER.size:])
        assert e.value.code == gpu_lib.E_INVALID, wrong
    t, _ = gpu_lib.archive_decode(buf)  # the library still works after the rejections
    assert t.info().n_voxels == tr.info().n_voxels


def test_archive_write_rejects_bad_descriptions(gpu_lib, fitted):
    tr, m = fitted["tree"], fitted["fp32"]
    for mask, explicit in ((0b110, False), (0b101, True), (0b001, False), (0, True), (8, True)):
        with pytest.raises(gpu_lib.NvdbError) as e:
            gpu_lib.archive_write(m, tr, mask, gpu_lib.STORE_F16, explicit_l1=explicit)
        assert e.value.code == gpu_lib.E_INVALID, (mask, explicit)
    # stored leaf masks: need the level-1 masks, exclude the level-0 classifier and patches
    for mask, explicit, patches in ((0b101, False, False), (0b011, True, False), (0b001, True, True)):
        with pytest.raises(gpu_lib.NvdbError) as e:
            gpu_lib.archive_write(m, tr, mask, gpu_lib.STORE_F16, explicit_l1=explicit, patches=patches,
                                  explicit_l0=True)
        assert e.value.code == gpu_lib.E_INVALID, (mask, explicit, patches)
    with pytest.raises(gpu_lib.NvdbError) as e:
        gpu_lib.archive_write(m, tr, 0b001, 7, explicit_l1=True)
    assert e.value.code == gpu_lib.E_INVALID
    fresh = gpu_lib.Model({0: NETS[0]}, precision=gpu_lib.FP32, domain_size=256, value_scale=3.0)
    with pytest.raises(gpu_lib.NvdbError) as e:
        gpu_lib.archive_write(fresh, tr, 0b001, gpu_lib.STORE_F16, explicit_l1=True)
    assert e.value.code == gpu_lib.E_STATE
