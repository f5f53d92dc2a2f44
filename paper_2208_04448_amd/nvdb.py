"""Thin ctypes binding of libnvdb (include/nvdb.h).

Argument marshalling only: every step of the encode/decode path runs in the
HIP kernels of libnvdb.so.  Torch provides device memory and the current
stream.  Importing this module fails loudly if the library has not been built.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnvdb.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("libnvdb.so is not built; run paper_2208_04448_amd/build.py (or __graft_entry__.build())")
_lib = C.CDLL(LIB_PATH)

OK, E_INVALID, E_NOMEM, E_DEVICE, E_NUMERIC, E_STATE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
SDF, FOG = 0, 1
NET_REGRESSOR, NET_L0, NET_L1, NET_TILE, MAX_NETS = 0, 1, 2, 3, 4
FP32, BF16 = 0, 1
STORE_F16, STORE_BF16 = 0, 1


class NvdbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("nvdb error %d: %s" % (code, msg))
        self.code = code


class ActiveRule(C.Structure):
    _fields_ = [("kind", C.c_int32), ("band_or_threshold", C.c_float)]


class TreeInfo(C.Structure):
    _fields_ = [("n_voxels", C.c_int64), ("n_leaves", C.c_int64), ("n_l1", C.c_int64), ("n_l2", C.c_int64),
                ("grid_origin", C.c_int32 * 3), ("grid_dims", C.c_int32 * 3),
                ("bytes_l2", C.c_int64), ("bytes_l1", C.c_int64), ("bytes_leaf_masks", C.c_int64),
                ("bytes_voxels", C.c_int64), ("n_tiles", C.c_int64)]


class NetDesc(C.Structure):
    _fields_ = [("width", C.c_int32), ("hidden", C.c_int32), ("n_freq", C.c_int32), ("n_out", C.c_int32),
                ("sin_freq", C.c_float)]


class ModelDesc(C.Structure):
    _fields_ = [("precision", C.c_int32), ("has_net", C.c_int32 * MAX_NETS), ("net", NetDesc * MAX_NETS),
                ("domain_lo", C.c_int32 * 3), ("domain_size", C.c_int32), ("value_scale", C.c_float)]


class FitDesc(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("seed", C.c_uint64), ("lr", C.c_float),
                ("lr_decay", C.c_float), ("lr_interval", C.c_int32), ("nets_mask", C.c_int32),
                ("idx_dev", C.c_void_p * MAX_NETS), ("idx_count", C.c_int64 * MAX_NETS), ("train_kernel_ms", C.c_void_p)]


class FrameReport(C.Structure):
    _fields_ = [("steps_run", C.c_int32 * MAX_NETS), ("final_loss", C.c_float * MAX_NETS)]


class L1Report(C.Structure):
    _fields_ = [("n_slots", C.c_int64), ("fp", C.c_int64), ("fn", C.c_int64), ("mismatch", C.c_int64)]


class TopologyReport(C.Structure):
    _fields_ = [("n_true", C.c_int64), ("n_pred", C.c_int64), ("fp", C.c_int64), ("fn", C.c_int64),
                ("n_common", C.c_int64), ("max_abs", C.c_double), ("rms", C.c_double)]


TUNE_MAX = 32
TRAIN_REGISTERS, TRAIN_ROWS = 0, 1


class TuneReport(C.Structure):
    _fields_ = [("chosen_g", C.c_int32), ("chosen_kernel", C.c_int32), ("n_candidates", C.c_int32),
                ("kernel", C.c_int32 * TUNE_MAX), ("g", C.c_int32 * TUNE_MAX), ("ms_per_step", C.c_float * TUNE_MAX)]


class DecodeTuneReport(C.Structure):
    _fields_ = [("n_candidates", C.c_int32), ("net", C.c_int32 * TUNE_MAX), ("waves", C.c_int32 * TUNE_MAX),
                ("tiles", C.c_int32 * TUNE_MAX), ("ms", C.c_float * TUNE_MAX), ("chosen", C.c_int32 * MAX_NETS)]


class ErrorReport(C.Structure):
    _fields_ = [("n", C.c_int64), ("max_abs", C.c_double), ("rms", C.c_double), ("iou", C.c_double),
                ("fp", C.c_int64), ("fn", C.c_int64)]


_P = C.c_void_p
class Subdomains(C.Structure):
    _fields_ = [("origin", C.c_int32 * 3), ("size", C.c_int32), ("halo", C.c_int32)]


class ArchiveDesc(C.Structure):
    _fields_ = [("nets_mask", C.c_int32), ("storage", C.c_int32), ("explicit_l1", C.c_int32), ("patches", C.c_int32),
                ("explicit_l0", C.c_int32)]


class ArchiveInfo(C.Structure):
    _fields_ = [("flags", C.c_int32), ("nets_mask", C.c_int32), ("rule_kind", C.c_int32), ("rule_thr", C.c_float),
                ("n_l2", C.c_int64), ("n_l1", C.c_int64), ("n_fp", C.c_int64), ("n_fn", C.c_int64),
                ("n_leaf", C.c_int64)]


_SIGS = {
    "nvdb_last_error": (C.c_char_p, []),
    "nvdb_abi_version": (C.c_int32, []),
    "nvdb_tree_build_dense": (C.c_int32, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(ActiveRule), _P,
                                          C.POINTER(_P)]),
    "nvdb_tree_build_sparse": (C.c_int32, [_P, _P, C.c_int64, C.POINTER(ActiveRule), _P, C.POINTER(_P)]),
    "nvdb_tree_get_info": (C.c_int32, [_P, C.POINTER(TreeInfo)]),
    "nvdb_tree_prune_tiles": (C.c_int32, [_P, _P, C.POINTER(_P)]),
    "nvdb_tree_export_tiles": (C.c_int32, [_P, _P, _P, _P]),
    "nvdb_decode_tiles": (C.c_int32, [_P, _P, C.c_int32, _P, _P]),
    "nvdb_errors_tiles": (C.c_int32, [_P, _P, C.POINTER(ErrorReport), _P]),
    "nvdb_query": (C.c_int32, [_P, _P, _P, C.c_int64, C.c_float, C.c_int64, _P, _P, _P]),
    "nvdb_topology_patches": (C.c_int32, [_P, _P, _P, C.c_int64, _P, C.c_int64, C.POINTER(C.c_int64),
                                          C.POINTER(C.c_int64), _P]),
    "nvdb_tree_export_l2": (C.c_int32, [_P, _P, _P]),
    "nvdb_subdomain_cells": (C.c_int32, [_P, C.POINTER(Subdomains), _P, C.c_int64, C.POINTER(C.c_int64), _P]),
    "nvdb_tree_subdomain": (C.c_int32, [_P, C.POINTER(Subdomains), C.POINTER(C.c_int32), _P, C.POINTER(_P)]),
    "nvdb_decode_moe": (C.c_int32, [C.POINTER(_P), _P, C.c_int32, C.POINTER(Subdomains), _P, _P, _P]),
    "nvdb_decode_moe_mask": (C.c_int32, [C.POINTER(_P), _P, C.c_int32, C.POINTER(Subdomains), _P, _P, _P]),
    "nvdb_decode_moe_l1": (C.c_int32, [C.POINTER(_P), _P, C.c_int32, C.POINTER(Subdomains), _P, _P, _P]),
    "nvdb_decode_moe_tiles": (C.c_int32, [C.POINTER(_P), _P, C.c_int32, C.POINTER(Subdomains), _P, _P, _P]),
    "nvdb_tree_export": (C.c_int32, [_P, _P, _P, _P, _P, _P, _P]),
    "nvdb_tree_free": (None, [_P]),
    "nvdb_model_create": (C.c_int32, [C.POINTER(ModelDesc), C.POINTER(_P)]),
    "nvdb_model_param_count": (C.c_int32, [_P, C.c_int32, C.POINTER(C.c_int64)]),
    "nvdb_model_set_params": (C.c_int32, [_P, C.c_int32, _P, C.c_int64]),
    "nvdb_model_get_params": (C.c_int32, [_P, C.c_int32, _P, C.c_int64]),
    "nvdb_model_get_params16": (C.c_int32, [_P, C.c_int32, C.c_int32, _P, C.c_int64]),
    "nvdb_model_set_params16": (C.c_int32, [_P, C.c_int32, C.c_int32, _P, C.c_int64]),
    "nvdb_model_set_encoding": (C.c_int32, [_P, C.c_int32, _P, C.c_int32]),
    "nvdb_model_get_opt_state": (C.c_int32, [_P, C.c_int32, _P, _P, C.c_int64, C.POINTER(C.c_int64)]),
    "nvdb_model_set_opt_state": (C.c_int32, [_P, C.c_int32, _P, _P, C.c_int64, C.c_int64]),
    "nvdb_model_free": (None, [_P]),
    "nvdb_fit": (C.c_int32, [_P, _P, C.POINTER(FitDesc), _P, _P]),
    "nvdb_fit_experts": (C.c_int32, [C.POINTER(_P), C.POINTER(_P), C.c_int32, C.POINTER(FitDesc), _P, _P]),
    "nvdb_fit_sequence": (C.c_int32, [_P, _P, C.c_int32, C.POINTER(FitDesc), C.POINTER(FitDesc), C.c_int32, _P, _P,
                                      _P, _P]),
    "nvdb_autotune": (C.c_int32, [_P, _P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(TuneReport), _P]),
    "nvdb_model_set_train_groups": (C.c_int32, [_P, C.c_int32]),
    "nvdb_model_set_train_kernel": (C.c_int32, [_P, C.c_int32]),
    "nvdb_autotune_decode": (C.c_int32, [_P, _P, C.c_int32, C.c_int32, C.POINTER(DecodeTuneReport), _P]),
    "nvdb_model_set_decode_shape": (C.c_int32, [_P, C.c_int32, C.c_int32]),
    "nvdb_decode": (C.c_int32, [_P, _P, _P, _P, _P]),
    "nvdb_decode_l1": (C.c_int32, [_P, _P, _P, _P]),
    "nvdb_decode_fp8": (C.c_int32, [_P, _P, _P, _P, _P]),
    "nvdb_decode_l1_fp8": (C.c_int32, [_P, _P, _P, _P]),
    "nvdb_errors": (C.c_int32, [_P, _P, _P, C.POINTER(ErrorReport), _P]),
    "nvdb_errors_l1": (C.c_int32, [_P, _P, C.POINTER(L1Report), _P]),
    "nvdb_decode_topology": (C.c_int32, [_P, _P, C.c_int32, C.POINTER(_P), _P]),
    "nvdb_errors_topology": (C.c_int32, [_P, _P, C.POINTER(TopologyReport), _P]),
    "nvdb_model_reserve_dev": (C.c_int32, [_P, C.c_int32, C.c_int64]),
    "nvdb_forward_dev": (C.c_int32, [_P, C.c_int32, _P, _P, C.c_int64, _P, _P]),
    "nvdb_backward_dev": (C.c_int32, [_P, C.c_int32, _P, _P, _P, C.c_int64, _P, _P]),
    "nvdb_forward_coords_dev": (C.c_int32, [_P, C.c_int32, _P, C.c_int64, _P, _P]),
    "nvdb_backward_coords_dev": (C.c_int32, [_P, C.c_int32, _P, _P, C.c_int64, _P, _P]),
    "nvdb_model_set_params_dev": (C.c_int32, [_P, C.c_int32, _P, C.c_int64, _P]),
    "nvdb_model_get_params_dev": (C.c_int32, [_P, C.c_int32, _P, C.c_int64, _P]),
    "nvdb_model_take_errors": (C.c_int32, [_P, C.POINTER(C.c_int64)]),
    "nvdb_subdomain_box": (C.c_int32, [C.POINTER(Subdomains), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]),
    "nvdb_query_noalloc": (C.c_int32, [_P, _P, _P, C.c_int64, C.c_float, C.c_int64, _P, _P, _P]),
    "nvdb_archive_write": (C.c_int32, [_P, _P, C.POINTER(ArchiveDesc), _P, C.c_int64, C.POINTER(C.c_int64), _P]),
    "nvdb_archive_decode": (C.c_int32, [_P, C.c_int64, C.POINTER(_P), C.POINTER(ArchiveInfo), _P]),
    "nvdb_sample_indices_dev": (C.c_int32, [C.c_uint64, C.c_int32, C.c_int64, C.c_int64, C.c_int64, _P, _P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


def _check(code):
    if code != OK:
        raise NvdbError(code, _lib.nvdb_last_error().decode())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _i3(v):
    return (C.c_int32 * 3)(*[int(a) for a in v])


def _index_tensor(t, name="idx"):
    """A population-index list as the library reads it: a contiguous 1-D int32 or
    uint32 CUDA tensor (an int64 tensor would be read as pairs of 32-bit words)."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype in (torch.int32, torch.uint32) and t.dim() == 1):
        raise NvdbError(E_INVALID, "%s must be a 1-D int32/uint32 CUDA tensor" % name)
    if not t.is_contiguous():
        raise NvdbError(E_INVALID, "%s must be contiguous" % name)
    return t


# ---------------------------------------------------------------------------- trees
class Tree:
    """Handle of a tree built on the device from a dense float32 grid (x-major)."""

    def __init__(self, grid, origin=(0, 0, 0), kind=SDF, band_or_threshold=3.0):
        import torch
        assert grid.is_cuda and grid.dtype == torch.float32 and grid.dim() == 3
        grid = grid.contiguous()
        h = C.c_void_p()
        rule = ActiveRule(kind, band_or_threshold)
        _check(_lib.nvdb_tree_build_dense(_ptr(grid), _i3(grid.shape), _i3(origin), C.byref(rule), _stream(),
                                          C.byref(h)))
        self.h = h
        self.kind = kind

    @classmethod
    def from_sparse(cls, ijk, values, kind=SDF, band_or_threshold=3.0):
        """Tree of a sparse voxel list: ijk int32 [n, 3] and values float32 [n], device tensors."""
        import torch
        assert ijk.is_cuda and values.is_cuda and ijk.dtype == torch.int32 and values.dtype == torch.float32
        ijk = ijk.contiguous().reshape(-1, 3)
        values = values.contiguous().reshape(-1)
        assert ijk.shape[0] == values.shape[0]
        h = C.c_void_p()
        rule = ActiveRule(kind, band_or_threshold)
        _check(_lib.nvdb_tree_build_sparse(_ptr(ijk), _ptr(values), values.numel(), C.byref(rule), _stream(),
                                           C.byref(h)))
        t = cls.__new__(cls)
        t.h = h
        t.kind = kind
        return t

    def export_l2(self):
        """Level-2 origins int32 [n_l2, 3] and child masks uint64 [n_l2, 512]."""
        n = self.info().n_l2
        o, c = np.zeros((n, 3), np.int32), np.zeros((n, 512), np.uint64)
        _check(_lib.nvdb_tree_export_l2(self.h, o.ctypes.data_as(C.c_void_p), c.ctypes.data_as(C.c_void_p)))
        return o, c

    def subdomain(self, origin, size, halo, cell):
        """Tree of this tree's voxels inside the widened box of `cell` (the expert's training set)."""
        g = Subdomains(_i3(origin), int(size), int(halo))
        h = C.c_void_p()
        _check(_lib.nvdb_tree_subdomain(self.h, C.byref(g), _i3(cell), _stream(), C.byref(h)))
        t = Tree.__new__(Tree)
        t.h = h
        t.kind = self.kind
        return t

    def info(self):
        i = TreeInfo()
        _check(_lib.nvdb_tree_get_info(self.h, C.byref(i)))
        return i

    def prune_tiles(self):
        """New tree with every full, constant leaf replaced by an active tile of its level-1 node."""
        h = C.c_void_p()
        _check(_lib.nvdb_tree_prune_tiles(self.h, _stream(), C.byref(h)))
        t = Tree.__new__(Tree)
        t.h = h
        t.kind = self.kind
        return t

    def export_tiles(self):
        """Active tiles: keys uint32 [T] (level-1 node << 12 | n1), values float32 [T],
        level-1 active-tile masks uint64 [n_l1, 64]."""
        i = self.info()
        k, v = np.zeros(i.n_tiles, np.uint32), np.zeros(i.n_tiles, np.float32)
        a = np.zeros((i.n_l1, 64), np.uint64)
        _check(_lib.nvdb_tree_export_tiles(self.h, *[o.ctypes.data_as(C.c_void_p) for o in (k, v, a)]))
        return k, v, a

    def export(self):
        i = self.info()
        L, N, L1 = i.n_leaves, i.n_voxels, i.n_l1
        out = dict(leaf_origin=np.zeros((L, 3), np.int32), leaf_mask=np.zeros((L, 8), np.uint64),
                   leaf_off=np.zeros(L + 1, np.uint32), values=np.zeros(N, np.float32),
                   l1_origin=np.zeros((L1, 3), np.int32), l1_child=np.zeros((L1, 64), np.uint64))
        _check(_lib.nvdb_tree_export(self.h, *[o.ctypes.data_as(C.c_void_p) for o in
                                               (out["leaf_origin"], out["leaf_mask"], out["leaf_off"], out["values"],
                                                out["l1_origin"], out["l1_child"])]))
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.nvdb_tree_free(self.h)
            self.h = None


# ---------------------------------------------------------------------------- models
class Model:
    """Handle of a set of NeuralVDB networks (regressor, level-0, level-1, tile values)."""

    def __init__(self, nets, precision=BF16, domain_lo=(0, 0, 0), domain_size=64, value_scale=1.0):
        """nets: {net_id: (width, hidden, n_freq, n_out[, sin_freq])}; sin_freq 0 (default) is ReLU."""
        d = ModelDesc()
        d.precision = precision
        for k, desc in nets.items():
            w, hh, m, c = desc[:4]
            d.has_net[k] = 1
            d.net[k] = NetDesc(w, hh, m, c, float(desc[4]) if len(desc) > 4 else 0.0)
        d.domain_lo = _i3(domain_lo)
        d.domain_size = int(domain_size)
        d.value_scale = float(value_scale)
        h = C.c_void_p()
        _check(_lib.nvdb_model_create(C.byref(d), C.byref(h)))
        self.h = h
        self.nets = dict(nets)
        self.precision = precision

    def param_count(self, net):
        n = C.c_int64()
        _check(_lib.nvdb_model_param_count(self.h, net, C.byref(n)))
        return n.value

    def set_params(self, net, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        _check(_lib.nvdb_model_set_params(self.h, net, a.ctypes.data_as(C.c_void_p), a.size))

    def get_params(self, net):
        a = np.zeros(self.param_count(net), np.float32)
        _check(_lib.nvdb_model_get_params(self.h, net, a.ctypes.data_as(C.c_void_p), a.size))
        return a

    def set_encoding(self, net, B):
        a = np.ascontiguousarray(B, dtype=np.float32)
        _check(_lib.nvdb_model_set_encoding(self.h, net, a.ctypes.data_as(C.c_void_p), a.shape[0]))

    def get_params16(self, net, kind):
        """Parameters rounded to 16 bits (STORE_F16 or STORE_BF16), uint16 numpy array."""
        out = np.zeros(self.param_count(net), np.uint16)
        _check(_lib.nvdb_model_get_params16(self.h, net, kind, out.ctypes.data_as(C.c_void_p), out.size))
        return out

    def set_params16(self, net, kind, p16):
        p16 = np.ascontiguousarray(p16, dtype=np.uint16)
        _check(_lib.nvdb_model_set_params16(self.h, net, kind, p16.ctypes.data_as(C.c_void_p), p16.size))

    def get_opt_state(self, net):
        n = self.param_count(net)
        m, v, s = np.zeros(n, np.float32), np.zeros(n, np.float32), C.c_int64()
        _check(_lib.nvdb_model_get_opt_state(self.h, net, m.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p),
                                             n, C.byref(s)))
        return m, v, s.value

    def set_opt_state(self, net, m, v, step):
        m = np.ascontiguousarray(m, np.float32)
        v = np.ascontiguousarray(v, np.float32)
        _check(_lib.nvdb_model_set_opt_state(self.h, net, m.ctypes.data_as(C.c_void_p),
                                             v.ctypes.data_as(C.c_void_p), m.size, int(step)))

    def fit(self, tree, steps, batch, nets_mask, seed=0, lr=1e-3, lr_decay=0.975, lr_interval=100, idx=None,
            return_losses=True, kernel_times=None):
        """Run `steps` Adam steps.  idx: optional {net: int32/uint32 device tensor} of sample indices.
        kernel_times: optional dict that receives 'train_kernel_ms' (HIP events around the launches)."""
        f = FitDesc()
        tk = C.c_float(0.0)
        if kernel_times is not None:
            f.train_kernel_ms = C.cast(C.pointer(tk), C.c_void_p)
        f.steps, f.batch, f.seed = steps, batch, seed
        f.lr, f.lr_decay, f.lr_interval, f.nets_mask = lr, lr_decay, lr_interval, nets_mask
        keep = []
        for k, t in (idx or {}).items():
            _index_tensor(t, "idx[%d]" % k)
            keep.append(t)
            f.idx_dev[k] = t.data_ptr()
            f.idx_count[k] = t.numel()
        losses = np.zeros((MAX_NETS, max(steps, 1)), np.float32) if return_losses else None
        _check(_lib.nvdb_fit(self.h, tree.h, C.byref(f),
                             losses.ctypes.data_as(C.c_void_p) if return_losses else None, _stream()))
        if kernel_times is not None:
            kernel_times["train_kernel_ms"] = tk.value
        return losses[:, :steps] if return_losses else None

    def autotune(self, tree, nets_mask, batch, reps=5):
        """Pick the training kernel and the work-groups per network for training steps
        of `batch` samples; returns (chosen G, {(kernel, G): ms per step}); the chosen
        kernel is in self.train_kernel."""
        r = TuneReport()
        _check(_lib.nvdb_autotune(self.h, tree.h, nets_mask, batch, reps, C.byref(r), _stream()))
        self.train_kernel = r.chosen_kernel
        return r.chosen_g, {(r.kernel[i], r.g[i]): r.ms_per_step[i] for i in range(r.n_candidates)}

    def set_train_kernel(self, kind):
        _check(_lib.nvdb_model_set_train_kernel(self.h, int(kind)))

    def autotune_decode(self, tree, nets_mask, reps=5):
        """Pick each network's decode tile shape; returns ({net: chosen index},
        [(net, waves, tiles, ms)])."""
        r = DecodeTuneReport()
        _check(_lib.nvdb_autotune_decode(self.h, tree.h, nets_mask, reps, C.byref(r), _stream()))
        cand = [(r.net[i], r.waves[i], r.tiles[i], r.ms[i]) for i in range(r.n_candidates)]
        return {k: r.chosen[k] for k in range(MAX_NETS) if (nets_mask >> k) & 1}, cand

    def set_decode_shape(self, net, index):
        _check(_lib.nvdb_model_set_decode_shape(self.h, int(net), int(index)))

    def set_train_groups(self, g):
        _check(_lib.nvdb_model_set_train_groups(self.h, int(g)))

    def fit_sequence(self, frames, cold, warm, nets_mask, use_graph=True, frame_params=True):
        """Warm-started fit of an animated sequence (one tree per frame).
        cold / warm: dicts with steps, batch, seed, lr and optionally lr_decay, lr_interval.
        Returns (reports: list of (steps_run[3], final_loss[3]) per frame,
        losses: float32[3][T], frame_params: device float32[n_frames][sum P] or None)."""
        import torch

        def desc(d):
            f = FitDesc()
            f.steps, f.batch, f.seed = d["steps"], d["batch"], d.get("seed", 0)
            f.lr, f.lr_decay, f.lr_interval = d["lr"], d.get("lr_decay", 0.975), d.get("lr_interval", 100)
            f.nets_mask = nets_mask
            return f
        fc, fw = desc(cold), desc(warm)
        n = len(frames)
        hs = (C.c_void_p * n)(*[t.h for t in frames])
        reps = (FrameReport * n)()
        T = cold["steps"] + n * warm["steps"]
        losses = np.zeros((MAX_NETS, T), np.float32)
        fp = None
        if frame_params:
            tot = sum(self.param_count(k) for k in range(MAX_NETS) if nets_mask & (1 << k))
            fp = torch.empty((n, tot), dtype=torch.float32, device="cuda")
        _check(_lib.nvdb_fit_sequence(self.h, hs, n, C.byref(fc), C.byref(fw), int(bool(use_graph)), reps,
                                      losses.ctypes.data_as(C.c_void_p), _ptr(fp), _stream()))
        out = [(list(r.steps_run), list(r.final_loss)) for r in reps]
        return out, losses, fp

    def decode(self, tree, values=True, masks=True, fp8=False):
        import torch
        i = tree.info()
        v = torch.empty(i.n_voxels, dtype=torch.float32, device="cuda") if values else None
        mk = torch.empty((i.n_leaves, 8), dtype=torch.int64, device="cuda") if masks else None
        f = _lib.nvdb_decode_fp8 if fp8 else _lib.nvdb_decode
        _check(f(self.h, tree.h, _ptr(v), _ptr(mk), _stream()))
        return v, mk

    def decode_l1(self, tree, fp8=False):
        import torch
        i = tree.info()
        out = torch.empty((i.n_l1, 4096), dtype=torch.uint8, device="cuda")
        f = _lib.nvdb_decode_l1_fp8 if fp8 else _lib.nvdb_decode_l1
        _check(f(self.h, tree.h, _ptr(out), _stream()))
        return out

    def decode_tiles(self, tree, fp8=False):
        """Tile value regressor at every active tile of `tree` (value units, device float32 [T])."""
        import torch
        out = torch.empty(tree.info().n_tiles, dtype=torch.float32, device="cuda")
        _check(_lib.nvdb_decode_tiles(self.h, tree.h, int(bool(fp8)), _ptr(out), _stream()))
        return out

    def decode_topology(self, upper, fp8=False):
        """Decode the lower tree levels below the level-1 nodes of `upper`; returns a new Tree."""
        h = C.c_void_p()
        _check(_lib.nvdb_decode_topology(self.h, upper.h, int(bool(fp8)), C.byref(h), _stream()))
        t = Tree.__new__(Tree)
        t.h = h
        t.kind = upper.kind
        return t

    def query(self, tree, q, background, batch=0, return_hits=False):
        """Online random access: values at float32 index-space positions q [n, 3]
        (device tensor); returns values (and uint8 hit flags)."""
        import torch
        q = q.contiguous().reshape(-1, 3)
        assert q.is_cuda and q.dtype == torch.float32
        n = q.shape[0]
        v = torch.empty(n, dtype=torch.float32, device=q.device)
        h = torch.empty(n, dtype=torch.uint8, device=q.device) if return_hits else None
        _check(_lib.nvdb_query(self.h, tree.h, _ptr(q), n, float(background), int(batch), _ptr(v), _ptr(h), _stream()))
        return (v, h) if return_hits else v

    def query_noalloc(self, tree, q, background, batch=0, values=None, hits=None):
        """nvdb_query_noalloc: the random access with no device allocation inside the
        library (static per-GPU scratch, batches of at most 65536).  Output tensors
        may be passed in; returns (values, hits)."""
        import torch
        q = q.contiguous().reshape(-1, 3)
        assert q.is_cuda and q.dtype == torch.float32
        n = q.shape[0]
        v = values if values is not None else torch.empty(n, dtype=torch.float32, device=q.device)
        _check(_lib.nvdb_query_noalloc(self.h, tree.h, _ptr(q), n, float(background), int(batch), _ptr(v), _ptr(hits),
                                       _stream()))
        return v, hits

    def reserve_dev(self, net, max_n):
        """Workspace for forward/backward calls of up to max_n samples (allocates once)."""
        _check(_lib.nvdb_model_reserve_dev(self.h, net, int(max_n)))

    def forward(self, net, tree, idx, out=None):
        """Network outputs [n, n_out] at population indices idx of `tree` (gathered and
        normalised in the kernel)."""
        import torch
        _index_tensor(idx)
        y = out if out is not None else torch.empty((idx.numel(), self.nets[net][3]), dtype=torch.float32,
                                                     device=idx.device)
        _check(_lib.nvdb_forward_dev(self.h, net, tree.h, _ptr(idx), idx.numel(), _ptr(y), _stream()))
        return y

    def backward(self, net, tree, idx, gy, out=None):
        """Summed parameter gradient of sum_i gy_i . y(idx_i) (canonical layout); needs reserve_dev."""
        import torch
        _index_tensor(idx)
        gy = gy.contiguous()
        assert gy.dtype == torch.float32 and gy.numel() == idx.numel() * self.nets[net][3]
        g = out if out is not None else torch.empty(self.param_count(net), dtype=torch.float32, device=idx.device)
        _check(_lib.nvdb_backward_dev(self.h, net, tree.h, _ptr(idx), _ptr(gy), idx.numel(), _ptr(g), _stream()))
        return g

    def forward_coords(self, net, x):
        """Network outputs at normalised coordinates x [n, 3] (device tensor)."""
        import torch
        x = x.contiguous()
        y = torch.empty((x.shape[0], self.nets[net][3]), dtype=torch.float32, device=x.device)
        _check(_lib.nvdb_forward_coords_dev(self.h, net, _ptr(x), x.shape[0], _ptr(y), _stream()))
        return y

    def backward_coords(self, net, x, gy):
        """Summed parameter gradient at normalised coordinates; needs reserve_dev."""
        import torch
        x, gy = x.contiguous(), gy.contiguous()
        g = torch.empty(self.param_count(net), dtype=torch.float32, device=x.device)
        _check(_lib.nvdb_backward_coords_dev(self.h, net, _ptr(x), _ptr(gy), x.shape[0], _ptr(g), _stream()))
        return g

    def set_params_dev(self, net, theta):
        """Load the canonical parameters from a float32 CUDA tensor (ordered on the current stream)."""
        import torch
        assert theta.is_cuda and theta.dtype == torch.float32 and theta.is_contiguous()
        _check(_lib.nvdb_model_set_params_dev(self.h, net, _ptr(theta), theta.numel(), _stream()))

    def get_params_dev(self, net):
        import torch
        t = torch.empty(self.param_count(net), dtype=torch.float32, device="cuda")
        _check(_lib.nvdb_model_get_params_dev(self.h, net, _ptr(t), t.numel(), _stream()))
        return t

    def take_errors(self):
        """Number of out-of-range sample indices read since the last call (synchronises)."""
        n = C.c_int64()
        _check(_lib.nvdb_model_take_errors(self.h, C.byref(n)))
        return n.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.nvdb_model_free(self.h)
            self.h = None


def errors(tree, values, pred_mask=None):
    r = ErrorReport()
    _check(_lib.nvdb_errors(tree.h, _ptr(values), _ptr(pred_mask), C.byref(r), _stream()))
    return dict(n=r.n, max_abs=r.max_abs, rms=r.rms, iou=r.iou, fp=r.fp, fn=r.fn)


def errors_tiles(tree, tile_values):
    r = ErrorReport()
    _check(_lib.nvdb_errors_tiles(tree.h, _ptr(tile_values), C.byref(r), _stream()))
    return dict(n=r.n, max_abs=r.max_abs, rms=r.rms)


def errors_l1(tree, classes):
    r = L1Report()
    _check(_lib.nvdb_errors_l1(tree.h, _ptr(classes), C.byref(r), _stream()))
    return dict(n_slots=r.n_slots, fp=r.fp, fn=r.fn, mismatch=r.mismatch)


def topology_patches(truth, pred):
    """False-positive and false-negative voxel lists (device int32 [n, 3], canonical order)."""
    import torch
    nfp, nfn = C.c_int64(), C.c_int64()
    _check(_lib.nvdb_topology_patches(truth.h, pred.h, None, 0, None, 0, C.byref(nfp), C.byref(nfn), _stream()))
    fp = torch.empty((nfp.value, 3), dtype=torch.int32, device="cuda")
    fn = torch.empty((nfn.value, 3), dtype=torch.int32, device="cuda")
    _check(_lib.nvdb_topology_patches(truth.h, pred.h, _ptr(fp), nfp.value, _ptr(fn), nfn.value, C.byref(nfp),
                                      C.byref(nfn), _stream()))
    return fp, fn


def archive_write(model, truth, nets_mask, storage=STORE_F16, explicit_l1=False, patches=None, explicit_l0=False):
    """Compact byte image (bytes) of the model's networks in nets_mask for the volume `truth`
    (patches default: stored unless the leaf masks are)."""
    if patches is None:
        patches = not explicit_l0
    d = ArchiveDesc(int(nets_mask), int(storage), int(bool(explicit_l1)), int(bool(patches)), int(bool(explicit_l0)))
    n = C.c_int64()
    _check(_lib.nvdb_archive_write(model.h, truth.h, C.byref(d), None, 0, C.byref(n), _stream()))
    buf = (C.c_uint8 * n.value)()
    _check(_lib.nvdb_archive_write(model.h, truth.h, C.byref(d), buf, n.value, C.byref(n), _stream()))
    return bytes(buf)


def archive_decode(data):
    """Tree decoded from an archive (bytes) and the archive's ArchiveInfo."""
    data = bytes(data)
    buf = (C.c_uint8 * max(len(data), 1)).from_buffer_copy(data or b"\0")
    h, info = C.c_void_p(), ArchiveInfo()
    _check(_lib.nvdb_archive_decode(buf, len(data), C.byref(h), C.byref(info), _stream()))
    t = Tree.__new__(Tree)
    t.h = h
    t.kind = info.rule_kind
    return t, info


def subdomain_cells(tree, origin, size, halo):
    """Cells (int32 [n, 3], ascending) whose core holds an active voxel of the tree."""
    g = Subdomains(_i3(origin), int(size), int(halo))
    n = C.c_int64()
    _check(_lib.nvdb_subdomain_cells(tree.h, C.byref(g), None, 0, C.byref(n), _stream()))
    out = np.zeros((n.value, 3), np.int32)
    _check(_lib.nvdb_subdomain_cells(tree.h, C.byref(g), out.ctypes.data_as(C.c_void_p), n.value, C.byref(n),
                                     _stream()))
    return out


def subdomain_box(origin, size, halo, cell):
    """Normalisation box of a cell's expert: (lower corner of the widened box, its edge)."""
    g = Subdomains(_i3(origin), int(size), int(halo))
    lo, d = (C.c_int32 * 3)(), C.c_int32()
    _check(_lib.nvdb_subdomain_box(C.byref(g), _i3(cell), lo, C.byref(d)))
    return list(lo), d.value


def decode_moe(experts, cells, origin, size, halo, tree):
    """Gate-weighted blend of the experts' regressors at the tree's active voxels (float32 [N], device)."""
    import torch
    cells = np.ascontiguousarray(np.asarray(cells, np.int32).reshape(-1, 3))
    assert len(cells) == len(experts)
    hs = (_P * len(experts))(*[e.h for e in experts])
    g = Subdomains(_i3(origin), int(size), int(halo))
    v = torch.empty(tree.info().n_voxels, dtype=torch.float32, device="cuda")
    _check(_lib.nvdb_decode_moe(hs, cells.ctypes.data_as(C.c_void_p), len(experts), C.byref(g), tree.h, _ptr(v),
                                _stream()))
    return v


def fit_experts(models, trees, steps, batch, nets_mask, seed=0, lr=1e-3, lr_decay=0.975, lr_interval=100,
                return_losses=False):
    """The fits of independent models (one per subdomain) on their trees, two at a time on the GPU."""
    assert len(models) == len(trees)
    f = FitDesc()
    f.steps, f.batch, f.seed = steps, batch, seed
    f.lr, f.lr_decay, f.lr_interval, f.nets_mask = lr, lr_decay, lr_interval, nets_mask
    hm = (_P * len(models))(*[m.h for m in models])
    ht = (_P * len(trees))(*[t.h for t in trees])
    losses = np.zeros((len(models), MAX_NETS, max(steps, 1)), np.float32) if return_losses else None
    _check(_lib.nvdb_fit_experts(hm, ht, len(models), C.byref(f),
                                 losses.ctypes.data_as(C.c_void_p) if return_losses else None, _stream()))
    return losses[:, :, :steps] if return_losses else None


def decode_moe_mask(experts, cells, origin, size, halo, tree):
    """Blended level-0 masks (int64 [n_leaves, 8] bit words, device) of the experts' classifiers."""
    import torch
    cells = np.ascontiguousarray(np.asarray(cells, np.int32).reshape(-1, 3))
    assert len(cells) == len(experts)
    hs = (_P * len(experts))(*[e.h for e in experts])
    g = Subdomains(_i3(origin), int(size), int(halo))
    mk = torch.empty((tree.info().n_leaves, 8), dtype=torch.int64, device="cuda")
    _check(_lib.nvdb_decode_moe_mask(hs, cells.ctypes.data_as(C.c_void_p), len(experts), C.byref(g), tree.h,
                                     _ptr(mk), _stream()))
    return mk


def decode_moe_l1(experts, cells, origin, size, halo, tree):
    """Blended level-1 classes (uint8 [n_l1, 4096], device) of the experts' level-1 classifiers."""
    import torch
    cells = np.ascontiguousarray(np.asarray(cells, np.int32).reshape(-1, 3))
    assert len(cells) == len(experts)
    hs = (_P * len(experts))(*[e.h for e in experts])
    g = Subdomains(_i3(origin), int(size), int(halo))
    out = torch.empty((tree.info().n_l1, 4096), dtype=torch.uint8, device="cuda")
    _check(_lib.nvdb_decode_moe_l1(hs, cells.ctypes.data_as(C.c_void_p), len(experts), C.byref(g), tree.h,
                                   _ptr(out), _stream()))
    return out


def decode_moe_tiles(experts, cells, origin, size, halo, tree):
    """Blended active-tile values (float32 [n_tiles], device) of the experts' tile value regressors."""
    import torch
    cells = np.ascontiguousarray(np.asarray(cells, np.int32).reshape(-1, 3))
    assert len(cells) == len(experts)
    hs = (_P * len(experts))(*[e.h for e in experts])
    g = Subdomains(_i3(origin), int(size), int(halo))
    out = torch.empty(tree.info().n_tiles, dtype=torch.float32, device="cuda")
    _check(_lib.nvdb_decode_moe_tiles(hs, cells.ctypes.data_as(C.c_void_p), len(experts), C.byref(g), tree.h,
                                      _ptr(out), _stream()))
    return out


def errors_topology(truth, pred):
    r = TopologyReport()
    _check(_lib.nvdb_errors_topology(truth.h, pred.h, C.byref(r), _stream()))
    return dict(n_true=r.n_true, n_pred=r.n_pred, fp=r.fp, fn=r.fn, n_common=r.n_common, max_abs=r.max_abs,
                rms=r.rms)


def sample_indices(seed, stream_id, step, n_pop, batch):
    import torch
    out = torch.empty(batch, dtype=torch.int32, device="cuda")
    _check(_lib.nvdb_sample_indices_dev(seed, stream_id, step, n_pop, batch, _ptr(out), _stream()))
    return out


# ---------------------------------------------------------------------------- autograd
def mlp_function():
    """torch.autograd.Function whose forward and backward are the fused HIP kernels.

    apply(model, net, tree, idx, theta) -> y [n, n_out]: the network with the
    canonical parameter tensor theta (float32 CUDA, P) at population indices idx
    of `tree`.  theta is loaded into the model on the current stream by both
    passes, so a torch optimiser can train it; its gradient is the fused
    backward kernel's, which recomputes the forward activations instead of
    storing them.  The model needs reserve_dev(net, n) for the backward."""
    import torch

    class NvdbMLP(torch.autograd.Function):
        @staticmethod
        def forward(ctx, model, net, tree, idx, theta):
            ctx.model, ctx.net, ctx.tree = model, net, tree
            ctx.save_for_backward(idx, theta)
            model.set_params_dev(net, theta.detach())
            return model.forward(net, tree, idx)

        @staticmethod
        def backward(ctx, gy):
            idx, theta = ctx.saved_tensors
            ctx.model.set_params_dev(ctx.net, theta.detach())
            g = ctx.model.backward(ctx.net, ctx.tree, idx, gy.float())
            return None, None, None, None, g

    return NvdbMLP
