#!/usr/bin/env python
"""Throughput of the NeuralVDB coordinate-MLP encode/decode on one MI355X.

Workload (one "step" = one pass of the whole hot path over the volume):
  * a narrow-band level set of a sphere displaced by 4-octave gradient noise
    (amplitude 0.1 R) in a 512^3 grid, band +-3 voxels, float32 values, already
    resident in HBM;
  * tree build (32^3 -> 16^3 -> 8^3 decomposition), fit of the voxel regressor
    and the level-0 mask classifier (4 x 128 ReLU MLPs, Fourier features m = 64,
    sigma = 10) for --fit-steps Adam steps of 2^18 samples per network,
    full decode (regressor at every active voxel, classifier at every voxel slot
    of every leaf) and the error report.
value = training samples (fwd+bwd, both networks) per second of whole-step time.
The same job runs once in the plain FP32 form for the equal-error comparison;
the FP64 oracle is timed on a bounded sample of the same workload on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded voxels/s + train samples/s (fwd+bwd), BF16 vs FP32 at fixed max error"
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3
BATCH = 1 << 18
W, H, M, C = 128, 4, 64, 1
BAND = 3.0
N_GRID = 512


def flops_fwd_bwd(K, W, H, C):
    """Algorithmic flops per sample: forward, weight gradients of all layers and
    input gradients of layers 2..H+1 (no padding, no recompute)."""
    mac_all = K * W + (H - 1) * W * W + W * C
    mac_dx = (H - 1) * W * W + W * C
    return 2 * mac_all + 2 * mac_all + 2 * mac_dx


def flops_fwd(K, W, H, C):
    return 2 * (K * W + (H - 1) * W * W + W * C)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fit-steps", type=int, default=2000)
    ap.add_argument("--skip-fp32", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (N=%d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2208_04448_amd import nvdb

    dev = "cuda"
    torch.cuda.init()
    t0 = time.time()
    grid = workloads.noise_sphere_sdf(N_GRID, center=(256.0, 256.0, 256.0), radius=200.0, amplitude=20.0,
                                      octaves=4, scale=64.0, seed=0, device=dev)
    torch.cuda.synchronize()
    print("volume generated in %.1fs" % (time.time() - t0), file=sys.stderr, flush=True)

    K = 2 * M
    B_enc = {0: workloads.ffm_matrix(M, 10.0, seed=11), 1: workloads.ffm_matrix(M, 10.0, seed=12)}
    theta0 = {0: workloads.init_params(K, W, H, C, seed=21), 1: workloads.init_params(K, W, H, C, seed=22)}
    P = len(theta0[0])
    zeros = np.zeros(P, np.float32)

    def make_model(prec):
        mdl = nvdb.Model({0: (W, H, M, C), 1: (W, H, M, C)}, precision=prec, domain_lo=(0, 0, 0),
                         domain_size=N_GRID, value_scale=BAND)
        for k in (0, 1):
            mdl.set_encoding(k, B_enc[k])
        return mdl

    def job(mdl, fit_steps, timing=None):
        """One pass of the hot path; returns (tree, values, masks, error report, losses)."""
        tree = nvdb.Tree(grid, (0, 0, 0), nvdb.SDF, BAND)
        for k in (0, 1):
            mdl.set_params(k, theta0[k])
            mdl.set_opt_state(k, zeros, zeros, 0)
        kt = {} if timing is not None else None
        losses = mdl.fit(tree, steps=fit_steps, batch=BATCH, nets_mask=3, seed=0, lr=1e-3, lr_decay=0.975,
                         lr_interval=100, kernel_times=kt)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        values, masks = mdl.decode(tree)
        e1.record()
        rep = nvdb.errors(tree, values, masks)
        if timing is not None:
            timing["train_kernel_ms"] = kt["train_kernel_ms"]
            timing["decode_ms"] = e0.elapsed_time(e1)
        return tree, values, masks, rep, losses

    bf = make_model(nvdb.BF16)
    for _ in range(args.warmup):
        job(bf, args.fit_steps)
    torch.cuda.synchronize()
    times, timing = [], {}
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        tree, values, masks, rep, losses = job(bf, args.fit_steps, timing)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    step_s = max(times)
    info = tree.info()
    N, L = info.n_voxels, info.n_leaves
    samples = 2 * BATCH * args.fit_steps
    value = samples / step_s

    f_train = flops_fwd_bwd(K, W, H, C)
    launch_flops = 2 * BATCH * f_train
    train_launch_s = timing["train_kernel_ms"] / 1e3 / args.fit_steps
    achieved = launch_flops / train_launch_s / 1e12
    decode_s = timing["decode_ms"] / 1e3
    dec_flops = (N + 512 * L) * flops_fwd(K, W, H, C)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "train samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "noise-displaced sphere SDF 512^3, band +-3 voxels; regressor + level-0 classifier "
                               "4x128 ReLU, Fourier features m=64 sigma=10; %d Adam steps x 2^18 samples per "
                               "network; tree build + fit + full decode + error report per step" % args.fit_steps,
                   "n_voxels": N, "n_leaves": L, "global_batch": BATCH, "fit_steps": args.fit_steps,
                   "parallelism": "single GPU"},
        "train_samples_per_s_fit_kernel": 2 * BATCH / train_launch_s,
        "decoded_voxels_per_s": N / decode_s,
        "decoded_slots_per_s": 512 * L / decode_s,
        "decode_ms": decode_s * 1e3,
        "decode_tflops": dec_flops / decode_s / 1e12,
        "bf16": {"max_abs_err_voxels": rep["max_abs"], "rms_err_voxels": rep["rms"], "iou": rep["iou"],
                 "l0_fp": rep["fp"], "l0_fn": rep["fn"], "final_loss": [float(losses[0, -1]), float(losses[1, -1])]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None,
                     "kernel": "k_train<bf16,128,4,128,1> (both networks per launch)",
                     "flops_per_launch": launch_flops, "avg_launch_ms": train_launch_s * 1e3},
    }
    print("bf16 jobs: %s s" % ["%.3f" % t for t in times], file=sys.stderr, flush=True)

    if not args.skip_fp32:
        print("fp32 form job (%d steps) ..." % args.fit_steps, file=sys.stderr, flush=True)
        fp = make_model(nvdb.FP32)
        t32 = {}
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, _, rep32, losses32 = job(fp, args.fit_steps, t32)
        torch.cuda.synchronize()
        s32 = time.perf_counter() - t
        a32 = launch_flops / (t32["train_kernel_ms"] / 1e3 / args.fit_steps) / 1e12
        out["fp32_form"] = {
            "train_samples_per_s": samples / s32, "ms_per_step": s32 * 1e3,
            "decoded_voxels_per_s": N / (t32["decode_ms"] / 1e3),
            "max_abs_err_voxels": rep32["max_abs"], "rms_err_voxels": rep32["rms"], "iou": rep32["iou"],
            "l0_fp": rep32["fp"], "l0_fn": rep32["fn"],
            "final_loss": [float(losses32[0, -1]), float(losses32[1, -1])],
            "train_tflops": a32, "train_frac_of_fp32_peak": a32 / PEAK_FP32_TFLOPS}
        out["bf16_vs_fp32"] = {"speedup_whole_step": out["value"] / out["fp32_form"]["train_samples_per_s"],
                               "bf16_reaches_fp32_max_err": rep["max_abs"] <= rep32["max_abs"],
                               "equal_steps": args.fit_steps}
        print("fp32 job: %.3f s" % s32, file=sys.stderr, flush=True)

    if not args.skip_cpu:
        print("cpu baseline (FP64 oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(grid)

    print(json.dumps(out), flush=True)


def cpu_baseline(grid):
    """The FP64 oracle on the host: 3 Adam steps of the regressor at 2^14 samples
    on the same volume, after building the oracle's own tree from the grid."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import workloads
    from oracle import fit as F, mlp, tree as T

    t = time.perf_counter()
    g = grid.cpu().numpy()
    ijk, vals = T.active_set_dense(g, (0, 0, 0), T.SDF, BAND)
    tr = T.build(ijk, vals)
    build_s = time.perf_counter() - t
    K = 2 * M
    shapes = mlp.layer_shapes(K, W, H, C)
    th = workloads.init_params(K, W, H, C, seed=21).astype(np.float64)
    B = workloads.ffm_matrix(M, 10.0, seed=11).astype(np.float64)
    steps, batch = 3, 1 << 14
    t = time.perf_counter()
    F.train(th, shapes, B, tr, "regressor", (0, 0, 0), N_GRID, T.SDF, BAND, steps=steps, batch=batch, seed=0)
    fit_s = time.perf_counter() - t
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    return {"value": steps * batch / fit_s, "unit": "train samples/s", "cores": int(threads), "kind": "oracle",
            "sample": "3 Adam steps x 2^14 samples of the 4x128 regressor on the same 512^3 volume, FP64 numpy "
                      "(oracle tree build of %d voxels took %.1f s, not counted)" % (len(vals), build_s)}


if __name__ == "__main__":
    main()
