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
The launch shape (work-groups per network) comes from the library's autotuner,
run once before the timed region.  The same job runs once in the plain FP32
form for the equal-error comparison; the FP64 oracle is timed on a bounded
sample of the same workload on the host.  Two further legs are reported beside
the headline (not in `value`): the warm-started sequence fit of 16 frames of an
advected water surface (1024 x 256 x 1024) and the two-level fog-volume decode
of a 1024^3 fBm cloud.
"""
import hashlib
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
    ap.add_argument("--skip-sequence", action="store_true")
    ap.add_argument("--skip-cloud", action="store_true")
    ap.add_argument("--skip-small", action="store_true")
    ap.add_argument("--skip-query", action="store_true")
    ap.add_argument("--skip-moe", action="store_true")
    ap.add_argument("--skip-tiles", action="store_true")
    ap.add_argument("--seq-frames", type=int, default=16)
    ap.add_argument("--seq-cap", type=int, default=2000)
    ap.add_argument("--seq-full-width", action="store_true",
                    help="sequence leg with the wet region at full width in every frame (no growth)")
    ap.add_argument("--train-groups", type=int, default=0,
                    help="work-groups per network; 0 runs the autotuner (profiling runs pin it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (N=%d requested)" % args.gpus,
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
    tune_tree = nvdb.Tree(grid, (0, 0, 0), nvdb.SDF, BAND)
    for k in (0, 1):
        bf.set_params(k, theta0[k])
    if args.train_groups > 0:
        tuned_g, tune_ms = args.train_groups, {}
        bf.set_train_groups(tuned_g)
        bf.train_kernel = nvdb.TRAIN_ROWS
    else:
        tuned_g, tune_ms = bf.autotune(tune_tree, nets_mask=3, batch=BATCH, reps=3)
    kname = {nvdb.TRAIN_REGISTERS: "registers", nvdb.TRAIN_ROWS: "rows"}
    dec_choice, dec_cands = bf.autotune_decode(tune_tree, nets_mask=3, reps=3)
    del tune_tree
    print("autotune: %s G=%d %s; decode %s" % (kname[bf.train_kernel], tuned_g,
                                               {"%s/%d" % (kname[k], g): round(t, 4) for (k, g), t in tune_ms.items()},
                                               dec_cands), file=sys.stderr, flush=True)
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
                     "frac": achieved / PEAK_BF16_TFLOPS,
                     "traffic": measured_traffic() if bf.train_kernel == nvdb.TRAIN_ROWS else None,
                     "kernel": ("k_train_rows<4>" if bf.train_kernel == nvdb.TRAIN_ROWS else "k_train<bf16,128,4,128,1>")
                     + " (BF16 4x128, both networks per launch)",
                     "flops_per_launch": launch_flops, "avg_launch_ms": train_launch_s * 1e3},
        "autotune": {"train_kernel": kname[bf.train_kernel], "work_groups_per_network": tuned_g,
                     "ms_per_step": {"%s/%d" % (kname[k], g): t for (k, g), t in tune_ms.items()},
                     "decode_shape": {str(k): dict(zip(("waves", "tiles_per_wave"),
                                                       [c for c in dec_cands if c[0] == k][i][1:3]))
                                      for k, i in dec_choice.items()},
                     "decode_ms": {"%d/%dx%d" % (n_, w_, t_): ms_ for n_, w_, t_, ms_ in dec_cands}},
    }
    print("bf16 jobs: %s s" % ["%.3f" % t for t in times], file=sys.stderr, flush=True)
    # FP8 form of the decode with the same (BF16-trained) weights
    bf.decode(tree, fp8=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    v8, m8 = bf.decode(tree, fp8=True)
    e1.record()
    torch.cuda.synchronize()
    d8 = e0.elapsed_time(e1) / 1e3
    rep8 = nvdb.errors(tree, v8, m8)
    out["fp8_decode"] = {"decoded_voxels_per_s": N / d8, "decode_ms": d8 * 1e3, "decode_tflops": dec_flops / d8 / 1e12,
                         "max_abs_err_voxels": rep8["max_abs"], "rms_err_voxels": rep8["rms"], "iou": rep8["iou"],
                         "l0_fp": rep8["fp"], "l0_fn": rep8["fn"],
                         "note": "e4m3 weights (per layer) and activations (per sample), FP32 accumulate; "
                                 "includes requantising the weights"}

    if not args.skip_fp32:
        print("fp32 form job (%d steps) ..." % args.fit_steps, file=sys.stderr, flush=True)
        fp = make_model(nvdb.FP32)
        for k in (0, 1):
            fp.set_params(k, theta0[k])
        tt = nvdb.Tree(grid, (0, 0, 0), nvdb.SDF, BAND)
        if args.train_groups > 0:
            g32 = args.train_groups
            fp.set_train_groups(g32)
        else:
            g32, _ = fp.autotune(tt, nets_mask=3, batch=BATCH, reps=2)
        del tt
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
            "train_tflops": a32, "train_frac_of_fp32_peak": a32 / PEAK_FP32_TFLOPS,
            "work_groups_per_network": g32}
        out["bf16_vs_fp32"] = {"speedup_whole_step": out["value"] / out["fp32_form"]["train_samples_per_s"],
                               "bf16_reaches_fp32_max_err": rep["max_abs"] <= rep32["max_abs"],
                               "equal_steps": args.fit_steps}
        # equal-error protocol: continue the BF16 fit in 250-step chunks (up to twice the
        # budget) until its max error is at most the FP32 form's
        if rep["max_abs"] > rep32["max_abs"]:
            steps, reached, e = args.fit_steps, False, rep
            t_extra = 0.0
            while steps < 2 * args.fit_steps:
                torch.cuda.synchronize()
                t = time.perf_counter()
                bf.fit(tree, steps=250, batch=BATCH, nets_mask=3, seed=0, lr=1e-3, lr_decay=0.975,
                       lr_interval=100, return_losses=False)  # the same schedule, continued
                torch.cuda.synchronize()
                t_extra += time.perf_counter() - t
                steps += 250
                v_, m_ = bf.decode(tree)
                e = nvdb.errors(tree, v_, m_)
                if e["max_abs"] <= rep32["max_abs"]:
                    reached = True
                    break
            out["bf16_vs_fp32"]["time_to_fp32_max_err"] = {
                "reached": reached, "bf16_steps": steps, "bf16_max_abs_err": e["max_abs"],
                "bf16_s": step_s + t_extra, "fp32_s": s32,
                "note": "BF16 job of fit_steps steps plus the continued steps, against the FP32 job"}
        print("fp32 job: %.3f s" % s32, file=sys.stderr, flush=True)

    # the networks stored at 16 bits (Sec. 4): decode error with binary16 weights
    saved = {k: bf.get_params(k) for k in (0, 1)}
    for k in (0, 1):
        bf.set_params16(k, nvdb.STORE_F16, bf.get_params16(k, nvdb.STORE_F16))
    v16, m16 = bf.decode(tree)
    r16 = nvdb.errors(tree, v16, m16)
    for k in (0, 1):
        bf.set_params(k, saved[k])
    out["fp16_storage"] = {"max_abs_err_voxels": r16["max_abs"], "rms_err_voxels": r16["rms"], "iou": r16["iou"],
                           "bytes_per_network": 2 * P,
                           "note": "both networks rounded to binary16 and decoded (BF16 form)"}
    if not args.skip_query:
        print("random-access leg ...", file=sys.stderr, flush=True)
        out["random_access"] = random_access_leg(bf, tree)
    moe_ctx = None
    if not args.skip_moe:
        print("sparse-domain-decomposition leg ...", file=sys.stderr, flush=True)
        out["moe"], moe_ctx = moe_leg(tree, bf, rep, args.fit_steps, tuned_g)
    c4_grads = None
    if not args.skip_small:
        print("small-network leg ...", file=sys.stderr, flush=True)
        out["small"], c4_grads = small_leg()
    if not args.skip_cpu:
        print("cpu baseline (FP64 oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(grid, moe_ctx, c4_grads)
    del grid, bf
    torch.cuda.empty_cache()
    if not args.skip_sequence:
        print("sequence leg ...", file=sys.stderr, flush=True)
        out["sequence"] = sequence_leg(args.seq_frames, args.seq_cap, tuned_g, args.seq_full_width)
        # the same sequence refined at the cold rate (Sec. 3.6 allows the same or a
        # smaller rate for the refinement): warm against cold only
        same = sequence_leg(args.seq_frames, args.seq_cap, tuned_g, args.seq_full_width, warm_lr=1e-3)
        out["sequence"]["warm_at_cold_rate"] = {k: same[k] for k in ("warm", "sequence_s", "warm_frames_hitting_cap",
                                                                     "warm_vs_cold")}
        out["sequence"]["warm_at_cold_rate"]["last_frame_rms"] = same["frames"][-1]["rms"]
        torch.cuda.empty_cache()
    if not args.skip_cloud:
        print("cloud leg ...", file=sys.stderr, flush=True)
        out["cloud"] = cloud_leg(args.fit_steps, tuned_g)
        torch.cuda.empty_cache()
    if not args.skip_tiles:
        print("active-tiles leg ...", file=sys.stderr, flush=True)
        out["tiles"] = tiles_leg(args.fit_steps // 2)
        torch.cuda.empty_cache()

    print(json.dumps(out), flush=True)


def tiles_leg(fit_steps, n=256, thr=0.05):
    """Fog with a saturated core (Sec. 3.3.1): leaves of constant density become active
    tiles; the level-1 classifier is ternary (leaf / active tile / inactive) and the tile
    value regressor encodes the tile values.  All four networks train together, then the
    lower levels are decoded top-down from the level-1 nodes."""
    import numpy as np
    import torch

    import workloads
    from paper_2208_04448_amd import nvdb
    c = n / 2.0
    grid = workloads.saturated_fog(n=n, center=(c, c + 3.0, c - 2.0), radius=0.44 * n, scale=n / 4.0, device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    full = nvdb.Tree(grid, (0, 0, 0), nvdb.FOG, thr)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t
    t = time.perf_counter()
    tree = full.prune_tiles()
    torch.cuda.synchronize()
    t_prune = time.perf_counter() - t
    fi, info = full.info(), tree.info()
    del full, grid
    nets = {0: (W, H, M, C), 1: (W, H, M, C), 2: (64, 4, 64, 3), 3: (64, 3, 32, 1)}
    mdl = nvdb.Model(nets, precision=nvdb.BF16, domain_lo=(0, 0, 0), domain_size=n, value_scale=1.0)
    sig = {0: 10.0, 1: 10.0, 2: 2.0, 3: 2.0}
    for k, (w_, h_, m_, c_) in nets.items():
        mdl.set_encoding(k, workloads.ffm_matrix(m_, sig[k], seed=60 + k))
        mdl.set_params(k, workloads.init_params(2 * m_, w_, h_, c_, seed=70 + k))
    mdl.set_train_groups(128)
    batch = 1 << 16
    torch.cuda.synchronize()
    t = time.perf_counter()
    losses = mdl.fit(tree, steps=fit_steps, batch=batch, nets_mask=15, seed=0, lr=1e-3, lr_decay=0.975,
                     lr_interval=100)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t
    vt = mdl.decode_tiles(tree)
    tile_err = nvdb.errors_tiles(tree, vt)
    l1 = nvdb.errors_l1(tree, mdl.decode_l1(tree))
    mdl.decode_topology(tree)
    torch.cuda.synchronize()
    t = time.perf_counter()
    pred = mdl.decode_topology(tree)
    torch.cuda.synchronize()
    t_dec = time.perf_counter() - t
    topo = nvdb.errors_topology(tree, pred)
    kt, vt_true, _ = tree.export_tiles()
    kp, vp, _ = pred.export_tiles()
    common, it, ip = np.intersect1d(kt, kp, return_indices=True)
    d = vp[ip].astype(np.float64) - vt_true[it]
    pi = pred.info()
    moe = tiles_moe(tree, n, fit_steps)
    return {"workload": "fog %d^3, density clamp(3 (1 - r/R) + 0.3 fbm, 0, 1), R = %.1f, threshold %.2f; leaves of "
                        "one density pruned to active tiles" % (n, 0.44 * n, thr),
            "n_voxels_before_pruning": fi.n_voxels, "n_leaves_before_pruning": fi.n_leaves,
            "n_voxels": info.n_voxels, "n_leaves": info.n_leaves, "n_tiles": info.n_tiles, "n_l1": info.n_l1,
            "build_ms": t_build * 1e3, "prune_ms": t_prune * 1e3,
            "networks": {"regressor": "4x128 m=64", "l0": "4x128 m=64", "l1": "4x64 m=64, 3 classes",
                         "tile": "3x64 m=32"},
            "fit_steps": fit_steps, "batch": batch, "fit_s": t_fit,
            "train_samples_per_s": 4 * batch * fit_steps / t_fit,
            "final_loss": [float(losses[k, -1]) for k in range(4)],
            "tile_err_true_topology": tile_err, "l1_report": l1,
            "decode_topology_ms": t_dec * 1e3,
            "decoded": {"n_voxels": pi.n_voxels, "n_leaves": pi.n_leaves, "n_tiles": pi.n_tiles,
                        "tiles_placed_right": int(len(common)), "tiles_fp": int(len(kp) - len(common)),
                        "tiles_fn": int(len(kt) - len(common)),
                        "tile_max_abs": float(np.abs(d).max()) if len(d) else 0.0,
                        "tile_rms": float(np.sqrt(np.mean(d * d))) if len(d) else 0.0,
                        "voxels": topo},
            "moe_tiles": moe}


def tiles_moe(tree, n, fit_steps, S=128, h=8):
    """The tile values under the sparse domain decomposition (Sec. 3.4): cells of
    edge S with an h-voxel halo; the experts whose widened box holds tiles (a tile's
    gates vanish outside the boxes that hold it, so the others take no part) each
    fit a tile value regressor on their own tiles, all in shared launches; then the
    blended decode of every tile and its error."""
    import torch

    import workloads
    from paper_2208_04448_amd import nvdb
    origin = (0, 0, 0)
    cells = nvdb.subdomain_cells(tree, origin, S, h)
    experts, subs, used = [], [], []
    for c in cells:
        sub = tree.subdomain(origin, S, h, c)
        if sub.info().n_tiles == 0:
            continue
        lo, D = nvdb.subdomain_box(origin, S, h, c)
        m = nvdb.Model({3: (64, 3, 32, 1)}, precision=nvdb.BF16, domain_lo=lo, domain_size=D, value_scale=1.0)
        m.set_encoding(3, workloads.ffm_matrix(32, 2.0, seed=63))
        m.set_params(3, workloads.init_params(64, 64, 3, 1, seed=73))
        experts.append(m)
        subs.append(sub)
        used.append(c)
    batch = 1 << 14
    torch.cuda.synchronize()
    t = time.perf_counter()
    nvdb.fit_experts(experts, subs, steps=fit_steps, batch=batch, nets_mask=8, seed=0, lr=1e-3, lr_decay=0.975,
                     lr_interval=100)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t
    v = nvdb.decode_moe_tiles(experts, used, origin, S, h, tree)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        v = nvdb.decode_moe_tiles(experts, used, origin, S, h, tree)
    torch.cuda.synchronize()
    t_dec = (time.perf_counter() - t) / 3
    return {"cells": "%d^3 cells, halo %d: %d kept, %d with tiles" % (S, h, len(cells), len(experts)),
            "expert_tiles": [s_.info().n_tiles for s_ in subs], "fit_steps": fit_steps, "batch": batch,
            "fit_s": t_fit, "blended_decode_ms": t_dec * 1e3, "tile_err": nvdb.errors_tiles(tree, v)}


def measured_traffic():
    """HBM bytes per launch of the timed train kernel from the committed rocprofv3
    counter summary, or None when the kernel's sources have changed since."""
    path = os.path.join(ROOT, "profiles", "k_train_rows_bf16_4x128_sphere512_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec.get("sources", []):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if not rec.get("sources") or rec.get("source_sha256") != h.hexdigest():
        return None
    return rec["traffic_bytes_per_launch"]


def sequence_leg(n_frames, cap, tuned_g, full_width=False, warm_lr=1e-4):
    """Warm-started fit of an animated sequence: frame 0 cold (2000 steps, lr 1e-3)
    then refit at 1e-4, later frames warm-started at 1e-4 until the batch loss is
    below frame 0's final loss (at most `cap` steps); then the last frame fitted
    cold for 2000 steps for comparison at an equal step budget."""
    import numpy as np
    import torch

    import workloads
    from paper_2208_04448_amd import nvdb
    t = time.perf_counter()
    trees, counts = [], []
    for f in range(n_frames):
        g = workloads.water_frame(f, n_frames=n_frames, device="cuda", **({"wet0": 1024.0} if full_width else {}))
        trees.append(nvdb.Tree(g, (0, 0, 0), nvdb.SDF, BAND))
        counts.append(int(trees[-1].info().n_voxels))
        del g
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    K = 2 * M
    th0 = {k: workloads.init_params(K, W, H, C, seed=31 + k) for k in (0, 1)}
    mdl = nvdb.Model({0: (W, H, M, C), 1: (W, H, M, C)}, precision=nvdb.BF16, domain_lo=(0, 0, 0),
                     domain_size=1024, value_scale=BAND)
    mdl.set_train_groups(tuned_g)
    for k in (0, 1):
        mdl.set_encoding(k, workloads.ffm_matrix(M, 10.0, seed=41 + k))
        mdl.set_params(k, th0[k])
    cold = dict(steps=2000, batch=BATCH, seed=0, lr=1e-3)
    warm = dict(steps=cap, batch=BATCH, seed=1, lr=warm_lr)
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps, Lseq, fp = mdl.fit_sequence(trees, cold, warm, nets_mask=3, use_graph=True)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t
    steps = [int(max(r[0][:2])) for r in reps]
    P = mdl.param_count(0)
    frames = []
    for f in range(n_frames):
        for k in (0, 1):
            mdl.set_params(k, fp[f, k * P:(k + 1) * P].cpu().numpy())
        v, mk = mdl.decode(trees[f])
        e = nvdb.errors(trees[f], v, mk)
        frames.append({"voxels": counts[f], "steps": [int(reps[f][0][0]), int(reps[f][0][1])],
                       "max_abs": e["max_abs"], "rms": e["rms"], "iou": e["iou"], "l0_fp": e["fp"], "l0_fn": e["fn"]})
    # the last frame from scratch, 2000 steps at the cold rate
    last = n_frames - 1
    for k in (0, 1):
        mdl.set_params(k, th0[k])
        mdl.set_opt_state(k, np.zeros(P, np.float32), np.zeros(P, np.float32), 0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    mdl.fit(trees[last], steps=2000, batch=BATCH, nets_mask=3, seed=7, lr=1e-3, return_losses=False)
    torch.cuda.synchronize()
    cold_s = time.perf_counter() - t
    v, mk = mdl.decode(trees[last])
    e = nvdb.errors(trees[last], v, mk)
    # warm against cold (Sec. 3.6): for sampled frames, the steps a cold fit (initial
    # weights, cold rate) needs until its batch loss, averaged over 100 steps, reaches
    # the warm-started frame's final loss (the same average), per network; cold fits
    # run in 250-step chunks up to three times the warm cap
    c0 = cold["steps"] + warm["steps"]
    warm_vs_cold = []
    for f in sorted({max(1, n_frames // 4), max(1, n_frames // 2), last}):
        seg = Lseq[:2, c0 + (f - 1) * cap: c0 + f * cap]
        target = seg[:, -100:].mean(axis=1)
        for k in (0, 1):
            mdl.set_params(k, th0[k])
            mdl.set_opt_state(k, np.zeros(P, np.float32), np.zeros(P, np.float32), 0)
        reached = [None, None]
        done = 0
        while done < 3 * cap and None in reached:
            Lc = mdl.fit(trees[f], steps=250, batch=BATCH, nets_mask=3, seed=11, lr=1e-3)
            done += 250
            for k in (0, 1):
                if reached[k] is None and Lc[k, -100:].mean() <= target[k]:
                    reached[k] = done
        warm_vs_cold.append({"frame": f, "warm_steps": [int(reps[f][0][0]), int(reps[f][0][1])],
                             "warm_final_loss": [float(t_) for t_ in target],
                             "cold_steps_to_warm_loss": reached, "cold_steps_run": done})
    total_steps = sum(steps)
    return {"workload": "advected noisy water surface 1024x256x1024, %d frames, band +-3, wet region %s; regressor + "
                        "level-0 classifier 4x128, FFM m=64 sigma=10, BF16, 2^18 samples per network per step"
                        % (n_frames, "at full width" if full_width else "growing from x < 288 to full width"),
            "frame_voxels_min_max": [min(counts), max(counts)], "frames_generated_s": gen_s,
            "cold": {"steps": 2000, "lr": 1e-3}, "warm": {"cap": cap, "lr": warm_lr},
            "sequence_s": seq_s, "steps_total": total_steps,
            "train_samples_per_s": 2 * BATCH * total_steps / seq_s,
            "warm_frames_hitting_cap": sum(1 for s_ in steps[1:] if s_ >= cap),
            "frames": frames,
            "last_frame_cold_2000": {"s": cold_s, "max_abs": e["max_abs"], "rms": e["rms"], "iou": e["iou"],
                                     "l0_fp": e["fp"], "l0_fn": e["fn"]},
            "warm_vs_cold": warm_vs_cold,
            "warm_vs_cold_note": "cold_steps_to_warm_loss null: not reached within cold_steps_run"}


def cloud_leg(fit_steps, tuned_g):
    """Fog volume: 1024^3 fBm cloud (6 octaves), active where the density exceeds
    0.55; voxel regressor 4x128 and level-1 node classifier 4x64 (3 classes) fitted
    for fit_steps steps, then the full decode of every active voxel and every
    leaf slot of the level-1 nodes."""
    import torch

    import workloads
    from paper_2208_04448_amd import nvdb
    t = time.perf_counter()
    g = workloads.fbm_cloud(1024, device="cuda")
    tree = nvdb.Tree(g, (0, 0, 0), nvdb.FOG, 0.55)
    del g
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    info = tree.info()
    mdl = nvdb.Model({0: (W, H, M, C), 2: (64, 4, M, 3)}, precision=nvdb.BF16, domain_lo=(0, 0, 0),
                     domain_size=1024, value_scale=1.0)
    mdl.set_train_groups(tuned_g)
    mdl.set_encoding(0, workloads.ffm_matrix(M, 10.0, seed=51))
    mdl.set_encoding(2, workloads.ffm_matrix(M, 10.0, seed=52))
    mdl.set_params(0, workloads.init_params(2 * M, W, H, C, seed=53))
    mdl.set_params(2, workloads.init_params(2 * M, 64, 4, 3, seed=54))
    torch.cuda.synchronize()
    t = time.perf_counter()
    mdl.fit(tree, steps=fit_steps, batch=BATCH, nets_mask=0b101, seed=0, lr=1e-3, return_losses=False)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    values, _ = mdl.decode(tree, values=True, masks=False)
    e1.record()
    classes = mdl.decode_l1(tree)
    e2.record()
    torch.cuda.synchronize()
    dec_s, l1_s = e0.elapsed_time(e1) / 1e3, e1.elapsed_time(e2) / 1e3
    rep = nvdb.errors(tree, values)
    r1 = nvdb.errors_l1(tree, classes)
    mdl.decode(tree, values=True, masks=False, fp8=True)
    torch.cuda.synchronize()
    e0.record()
    values8, _ = mdl.decode(tree, values=True, masks=False, fp8=True)
    e1.record()
    classes8 = mdl.decode_l1(tree, fp8=True)
    e2.record()
    torch.cuda.synchronize()
    dec8_s, l18_s = e0.elapsed_time(e1) / 1e3, e1.elapsed_time(e2) / 1e3
    rep8 = nvdb.errors(tree, values8)
    r18 = nvdb.errors_l1(tree, classes8)
    # full decode of the lower levels: level-1 classes -> leaves -> regressor with the active rule
    N, L1 = int(info.n_voxels), int(info.n_l1)
    topo = {}
    for name, f8 in (("bf16", False), ("fp8", True)):
        mdl.decode_topology(tree, fp8=f8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pred = mdl.decode_topology(tree, fp8=f8)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rt = nvdb.errors_topology(tree, pred)
        pi = pred.info()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fpl, fnl = nvdb.topology_patches(tree, pred)
        torch.cuda.synchronize()
        patch_s = time.perf_counter() - t0
        # storage (Sec. 4, Tab. memory_cost accounting): the explicit tree against the
        # [Hash,5,NN(4),NN(3)] form with 16-bit networks and 12-byte patch coordinates
        explicit = int(info.bytes_l2 + info.bytes_l1 + info.bytes_leaf_masks + info.bytes_voxels)
        nets_b = 2 * (mdl.param_count(0) + mdl.param_count(2))
        neural = int(info.bytes_l2) + nets_b + 12 * (len(fpl) + len(fnl))
        topo[name] = {"s": dt, "predicted_leaves": int(pi.n_leaves), "predicted_voxels": int(pi.n_voxels),
                      "slots_evaluated_per_s": (4096 * L1 + 512 * int(pi.n_leaves)) / dt,
                      "fp": rt["fp"], "fn": rt["fn"], "n_common": rt["n_common"], "rms_err_common": rt["rms"],
                      "max_abs_err_common": rt["max_abs"], "patches_s": patch_s,
                      "bytes_explicit": explicit, "bytes_neural_lossless_topology": neural,
                      "compression_ratio": explicit / neural}
        del pred, fpl, fnl
    # the stored objects: compact archives written and decoded back to the true topology,
    # [Hash,5,4,NN(3)] (level-1 and leaf masks stored, the regressor for the values) and
    # [Hash,5,NN(4),NN(3)] without a level-0 classifier (level-1 classifier + regressor
    # with the active rule, patches); 16-bit weights
    explicit = int(info.bytes_l2 + info.bytes_l1 + info.bytes_leaf_masks + info.bytes_voxels)
    archive = {"bytes_explicit": explicit}
    for name, mask, kw in (("hash54nn3", 0b001, dict(explicit_l1=True, explicit_l0=True)),
                           ("hash5nn4nn3", 0b101, dict(explicit_l1=False, patches=True))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        blob = nvdb.archive_write(mdl, tree, mask, nvdb.STORE_F16, **kw)
        wr_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        back, ainfo = nvdb.archive_decode(blob)
        torch.cuda.synchronize()
        rd_s = time.perf_counter() - t0
        ra = nvdb.errors_topology(tree, back)
        archive[name] = {"bytes": len(blob), "compression_ratio": explicit / len(blob),
                         "patches": int(ainfo.n_fp + ainfo.n_fn), "write_s": wr_s, "decode_s": rd_s,
                         "decoded_fp": ra["fp"], "decoded_fn": ra["fn"], "decoded_rms_err": ra["rms"],
                         "decoded_max_abs_err": ra["max_abs"], "decoded_voxels_per_s": N / rd_s}
        del back, blob
    # sparse domain decomposition in the paper's cell range (Sec. 3.4: 512 to 2048):
    # 512^3 cells with an 8-voxel halo, one BF16 regressor per kept cell fitted as
    # long as the single regressor, blended decode against the single decode
    size, halo = 512, 8
    cells = nvdb.subdomain_cells(tree, (0, 0, 0), size, halo)
    experts, subs = [], []
    for c in cells:
        subs.append(tree.subdomain((0, 0, 0), size, halo, c))
        lo, D = nvdb.subdomain_box((0, 0, 0), size, halo, c)
        e = nvdb.Model({0: (W, H, M, C)}, precision=nvdb.BF16, domain_lo=lo, domain_size=D, value_scale=1.0)
        e.set_encoding(0, workloads.ffm_matrix(M, 10.0, seed=51))
        e.set_params(0, workloads.init_params(2 * M, W, H, C, seed=53))
        e.set_train_groups(tuned_g)
        experts.append(e)
    pairs = sum(int(s_.info().n_voxels) for s_ in subs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nvdb.fit_experts(experts, subs, steps=fit_steps, batch=BATCH, nets_mask=1, seed=0, lr=1e-3, lr_decay=0.975,
                     lr_interval=100)
    torch.cuda.synchronize()
    moe_fit_s = time.perf_counter() - t0
    del subs
    vm = nvdb.decode_moe(experts, cells, (0, 0, 0), size, halo, tree)
    rm = nvdb.errors(tree, vm)
    del vm
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vm = nvdb.decode_moe(experts, cells, (0, 0, 0), size, halo, tree)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        del vm
    moe_dec_s = sorted(ts)[1]
    moe = {"subdomain_size": size, "halo": halo, "experts": len(cells), "routed_pairs_per_voxel": pairs / N,
           "fit_s": moe_fit_s, "train_samples_per_s": len(cells) * fit_steps * BATCH / moe_fit_s,
           "blend_decode_ms": moe_dec_s * 1e3, "blend_voxels_per_s": N / moe_dec_s,
           "rms_err": rm["rms"], "max_abs_err": rm["max_abs"],
           "single_network": {"rms_err": rep["rms"], "max_abs_err": rep["max_abs"], "decode_ms": dec_s * 1e3}}
    del experts
    return {"workload": "fBm cloud 1024^3 (6 octaves, lacunarity 2, gain 0.5), active where density > 0.55; "
                        "voxel regressor 4x128 + level-1 classifier 4x64 (3 classes), FFM m=64 sigma=10, BF16; "
                        "%d steps x 2^18 samples per network" % fit_steps,
            "n_voxels": N, "n_leaves": int(info.n_leaves), "n_l1": L1, "generated_s": gen_s, "fit_s": fit_s,
            "decoded_voxels_per_s": N / dec_s, "decode_ms": dec_s * 1e3,
            "decode_tflops": N * flops_fwd(2 * M, W, H, C) / dec_s / 1e12,
            "l1_slots_per_s": 4096 * L1 / l1_s, "l1_decode_ms": l1_s * 1e3,
            "rms_err": rep["rms"], "max_abs_err": rep["max_abs"],
            "l1": {"n_slots": r1["n_slots"], "fp": r1["fp"], "fn": r1["fn"], "mismatch": r1["mismatch"]},
            "topology_decode": topo, "archive": archive, "moe_512": moe,
            "fp8": {"decoded_voxels_per_s": N / dec8_s, "decode_ms": dec8_s * 1e3,
                    "decode_tflops": N * flops_fwd(2 * M, W, H, C) / dec8_s / 1e12,
                    "frac_of_fp8_peak": N * flops_fwd(2 * M, W, H, C) / dec8_s / 1e12 / 5000.0,
                    "l1_slots_per_s": 4096 * L1 / l18_s, "rms_err": rep8["rms"], "max_abs_err": rep8["max_abs"],
                    "l1": {"fp": r18["fp"], "fn": r18["fn"], "mismatch": r18["mismatch"]}}}


def moe_leg(tree, single, rep_single, fit_steps, tuned_g, size=256, halo=8, reps=3):
    """Sparse domain decomposition (Sec. 3.4, eq. moe) of the 512^3 volume into
    256^3 subdomains with an 8-voxel halo: one BF16 regressor and one level-0
    classifier per kept cell, each fitted for fit_steps steps on its widened box,
    then the gate-weighted blended decode of every active voxel (timed against
    the single network's regressor decode of the same tree, median of `reps`
    after one warm-up) and the blended level-0 masks."""
    import numpy as np
    import torch

    import workloads
    from paper_2208_04448_amd import nvdb

    origin = (0, 0, 0)
    cells = nvdb.subdomain_cells(tree, origin, size, halo)
    K = 2 * M
    B0 = workloads.ffm_matrix(M, 10.0, seed=11)
    B1 = workloads.ffm_matrix(M, 10.0, seed=12)
    th0 = workloads.init_params(K, W, H, C, seed=21)
    th1 = workloads.init_params(K, W, H, C, seed=22)
    experts, subs, n_sub = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in cells:
        sub = tree.subdomain(origin, size, halo, c)
        subs.append(sub)
        n_sub.append(sub.info().n_voxels)
        lo, D = nvdb.subdomain_box(origin, size, halo, c)
        mdl = nvdb.Model({0: (W, H, M, C), 1: (W, H, M, C)}, precision=nvdb.BF16, domain_lo=lo, domain_size=D,
                         value_scale=BAND)
        mdl.set_encoding(0, B0)
        mdl.set_params(0, th0)
        mdl.set_encoding(1, B1)
        mdl.set_params(1, th1)
        if tuned_g:
            mdl.set_train_groups(tuned_g)
        experts.append(mdl)
    torch.cuda.synchronize()
    t_split = time.perf_counter() - t0
    t0 = time.perf_counter()
    nvdb.fit_experts(experts, subs, steps=fit_steps, batch=BATCH, nets_mask=3, seed=0, lr=1e-3, lr_decay=0.975,
                     lr_interval=100)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0

    def timed(f):
        f()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            f()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    values = nvdb.decode_moe(experts, cells, origin, size, halo, tree)
    masks = nvdb.decode_moe_mask(experts, cells, origin, size, halo, tree)
    r = nvdb.errors(tree, values, masks)
    n = tree.info().n_voxels
    t_moe = timed(lambda: nvdb.decode_moe(experts, cells, origin, size, halo, tree))
    t_one = timed(lambda: single.decode(tree, masks=False))
    pairs = sum(n_sub)
    ctx = {"cells": cells, "origin": origin, "size": size, "halo": halo,
           "experts": [(e.get_params(0), nvdb.subdomain_box(origin, size, halo, c)) for e, c in zip(experts, cells)]}
    return {"subdomain_size": size, "halo": halo, "experts": len(cells), "voxels": n,
            "routed_pairs_per_voxel": float(sum(n_sub)) / n,
            "split_s": t_split, "fit_s": t_fit, "steps_per_expert": fit_steps,
            "train_samples_per_s": 2 * len(cells) * fit_steps * BATCH / t_fit,
            "blend_decode_ms": t_moe * 1e3, "blend_voxels_per_s": n / t_moe,
            "blend_tflops_whole_call": pairs * flops_fwd(2 * M, W, H, C) / t_moe / 1e12,
            "single_decode_ms": t_one * 1e3, "single_voxels_per_s": n / t_one,
            "max_abs_err_voxels": r["max_abs"], "rms_err_voxels": r["rms"], "iou": r["iou"],
            "l0_fp": r["fp"], "l0_fn": r["fn"],
            "single_network": {"max_abs_err_voxels": rep_single["max_abs"], "rms_err_voxels": rep_single["rms"],
                               "iou": rep_single["iou"], "l0_fp": rep_single["fp"], "l0_fn": rep_single["fn"]},
            "note": "one regressor and one level-0 classifier per kept 256^3 cell, each fitted for the single "
                    "network's step count on its widened box (nvdb_fit_experts); split = subdomain trees + models; "
                    "blended decode = routing + one forward launch per expert + blend (values), wall clock; "
                    "l0_fp / l0_fn from the blended level-0 masks"}, ctx


def random_access_leg(model, tree, n=1 << 20, batch=1 << 16, reps=5):
    """Online random access (the tree decides, the regressor runs on active-voxel
    hits only) of n uniform positions in the 512^3 box, in batches of 2^16 as the
    paper measures it, against the pure network (the regressor on every
    position); median of `reps` after one warm-up, the trained BF16 networks."""
    import numpy as np
    import torch

    g = torch.Generator(device="cuda").manual_seed(5)
    q = torch.rand((n, 3), generator=g, device="cuda") * float(N_GRID)
    x = (q / float(N_GRID)).contiguous()

    def timed(f):
        f()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            f()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    _, hits = model.query(tree, q, background=BAND, batch=batch, return_hits=True)
    t_q = timed(lambda: model.query(tree, q, background=BAND, batch=batch))
    t_q1 = timed(lambda: model.query(tree, q, background=BAND, batch=0))
    t_nn = timed(lambda: model.forward_coords(0, x))
    return {"queries": n, "batch": batch, "hit_fraction": float(hits.float().mean().item()),
            "query_ms": t_q * 1e3, "queries_per_s": n / t_q, "query_ms_one_pass": t_q1 * 1e3,
            "pure_network_ms": t_nn * 1e3,
            "note": "uniform positions in the grid box; batches of 2^16 cost 4 launches each; one pass = all "
                    "queries in one batch; pure network = regressor on every position (one launch)"}


def small_leg(reps=5):
    """The 64^3 sphere with the 3x64 PE-6 networks: latency of the one-epoch job
    (tree build, 11 regressor + 33 level-0 classifier steps of 4096 samples over
    seeded permutations, full decode, error report), and fwd+bwd throughput at
    batch 2^22 through the autograd function (forward, then the fused backward
    that recomputes the activations), median of `reps` after one warm-up."""
    import numpy as np
    import torch

    import workloads
    from paper_2208_04448_amd import nvdb

    grid = workloads.sphere_sdf(device="cuda")
    B = workloads.pe_matrix(6)
    th0 = {0: workloads.init_params(36, 64, 3, 1, seed=0), 1: workloads.init_params(36, 64, 3, 1, seed=1)}
    perm = {0: workloads.epoch_permutation(43878, seed=5), 1: workloads.epoch_permutation(512 * 257, seed=6)}
    idx = {k: torch.from_numpy(perm[k].astype(np.int32)).cuda() for k in (0, 1)}
    steps = {0: 11, 1: 33}
    zeros = np.zeros(len(th0[0]), np.float32)
    res = {"workload": "64^3 sphere SDF (r 24, band +-3, 43,878 voxels, 257 leaves); regressor + level-0 "
                       "classifier 3x64, PE-6 (K 36)"}
    c4_grads = {}
    for name, prec in (("fp32", nvdb.FP32), ("bf16", nvdb.BF16)):
        model = nvdb.Model({0: (64, 3, 18, 1), 1: (64, 3, 18, 1)}, precision=prec, domain_size=64, value_scale=BAND)
        for k in (0, 1):
            model.set_encoding(k, B)

        def one_epoch():
            tree = nvdb.Tree(grid, (0, 0, 0), nvdb.SDF, BAND)
            for k in (0, 1):
                model.set_params(k, th0[k])
                model.set_opt_state(k, zeros, zeros, 0)
                model.fit(tree, steps=steps[k], batch=4096, nets_mask=1 << k, idx={k: idx[k]}, return_losses=False)
            v, m = model.decode(tree)
            return nvdb.errors(tree, v, m)

        one_epoch()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            rep = one_epoch()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        # C4: batch 2^22 i.i.d. voxel samples, MSE against the targets; the kernels gather
        # and normalise the samples from their population indices
        n = 1 << 22
        tree = nvdb.Tree(grid, (0, 0, 0), nvdb.SDF, BAND)
        ii = nvdb.sample_indices(0, 0, 0, 43878, n)
        vals = torch.from_numpy(tree.export()["values"] / BAND).cuda()
        ts_ = vals[ii.long()].contiguous()
        model.reserve_dev(0, n)
        Fn = nvdb.mlp_function()
        theta = torch.from_numpy(th0[0]).cuda().requires_grad_(True)

        def fwd_bwd():
            theta.grad = None
            y = Fn.apply(model, 0, tree, ii, theta)
            ((y[:, 0] - ts_) ** 2).mean().backward()

        fwd_bwd()
        tb = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fwd_bwd()
            torch.cuda.synchronize()
            tb.append(time.perf_counter() - t)
        # gradient of the same loss over the batch's first 2^16 samples, for the check
        # against the oracle in the cpu_baseline leg
        nc = 1 << 16
        theta.grad = None
        y = Fn.apply(model, 0, tree, ii[:nc].contiguous(), theta)
        ((y[:, 0] - ts_[:nc]) ** 2).mean().backward()
        c4_grads[name] = theta.grad.detach().cpu().numpy().astype(np.float64)
        med = float(np.median(tb))
        res[name] = {"one_epoch_job_ms": float(np.median(ts)) * 1e3, "max_abs_err_voxels": rep["max_abs"],
                     "rms_err_voxels": rep["rms"], "iou": rep["iou"],
                     "batch_2_22_fwd_bwd_ms": med * 1e3, "batch_2_22_samples_per_s": n / med,
                     "batch_2_22_tflops": n * flops_fwd_bwd(36, 64, 3, 1) / med / 1e12}
        del model
    return res, c4_grads


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def c4_gradient_check(c4_grads):
    """The C4 gradient check against the FP64 oracle: the GPU gradients of the MSE
    over the first 2^16 samples of the C4 batch (i.i.d. voxel samples of the 64^3
    sphere, 3x64 PE-6 regressor) against the oracle's analytic gradient, per tensor
    and on 256 weights drawn with seed 0; and the oracle's analytic gradient against
    central finite differences (h = 1e-3, FP64) of the loss over the first 2^10
    samples on the same 256 weights.  A weight whose +-h perturbation moves any
    hidden pre-activation across zero (a ReLU kink, where the difference quotient
    is not the derivative) is reported apart.  The full 2^22 batch is compared in
    the parity tests."""
    import numpy as np

    import workloads
    from oracle import fit as F, mlp, sampler as S, tree as T

    t0 = time.perf_counter()
    v = workloads.sphere_sdf().numpy()
    ot = T.build(*T.active_set_dense(v, (0, 0, 0), T.SDF, BAND))
    shapes = mlp.layer_shapes(36, 64, 3, 1)
    B = workloads.pe_matrix(6).astype(np.float64)
    th = workloads.init_params(36, 64, 3, 1, seed=0).astype(np.float64)
    params = mlp.unflatten(th, shapes)
    n = 1 << 16
    idx = S.iid_indices(0, 0, 0, 1 << 22, len(ot["values"]))[:n]
    x, t = F.net_inputs(ot, "regressor", idx, (0, 0, 0), 64, T.SDF, BAND)
    yo, cache = mlp.forward(params, mlp.encode(x, B))
    go = mlp.flatten(mlp.backward(params, cache, 2.0 * (yo[:, 0] - t)[:, None] / n))
    pick = np.random.default_rng(0).choice(len(th), 256, replace=False)
    out = {"samples": n, "weights_sampled": 256}
    for name, g in c4_grads.items():
        rel = np.abs(g[pick] - go[pick]) / np.maximum(np.abs(go[pick]), 1e-12)
        a, te = 0, []
        for o, i_ in shapes:
            for m_ in (o * i_, o):
                te.append(float(np.max(np.abs(g[a:a + m_] - go[a:a + m_])) / max(np.max(np.abs(go[a:a + m_])), 1e-30)))
                a += m_
        out["gpu_%s_vs_oracle" % name] = {"sampled_max_rel": float(np.max(rel)),
                                           "sampled_median_rel": float(np.median(rel)),
                                           "max_tensor_elementwise": max(te)}
    nf, h = 1 << 10, 1e-3
    z0 = mlp.encode(x[:nf], B)
    ts = t[:nf]

    def run(theta):
        y, c = mlp.forward(mlp.unflatten(theta, shapes), z0)
        return float(np.mean((y[:, 0] - ts) ** 2)), [c[i] > 0 for i in range(1, len(c), 2)]
    l0, pat0 = run(th)
    yo, cache = mlp.forward(params, z0)
    ga = mlp.flatten(mlp.backward(params, cache, 2.0 * (yo[:, 0] - ts)[:, None] / nf))
    rel, kink = np.empty(len(pick)), np.zeros(len(pick), bool)
    for q, k in enumerate(pick):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        (lp, pp), (lm, pm) = run(tp), run(tm)
        kink[q] = any(np.any(a != b) or np.any(a != c) for a, b, c in zip(pat0, pp, pm))
        rel[q] = abs((lp - lm) / (2 * h) - ga[k]) / max(abs(ga[k]), 1e-12)
    out["oracle_vs_fd"] = {"samples": nf, "h": h, "smooth_weights": int(np.sum(~kink)),
                           "smooth_max_rel": float(np.max(rel[~kink])) if np.any(~kink) else None,
                           "smooth_median_rel": float(np.median(rel[~kink])) if np.any(~kink) else None,
                           "kink_weights": int(np.sum(kink)),
                           "kink_max_rel": float(np.max(rel[kink])) if np.any(kink) else None}
    out["seconds"] = time.perf_counter() - t0
    return out


def cpu_baseline(grid, moe_ctx=None, c4_grads=None):
    """The FP64 oracle on the host: Adam steps of the 4x128 regressor at 2^14
    samples and the decode of sampled voxels on the same volume, on all host
    cores (numpy's BLAS threads) and on one thread; with the experts of the
    decomposition leg, the oracle's blended decode of 2^14 sampled voxels; with
    the small leg's gradients, the C4 gradient check."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

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
    batch = 1 << 14

    def rates(steps, nd):
        t = time.perf_counter()
        F.train(th, shapes, B, tr, "regressor", (0, 0, 0), N_GRID, T.SDF, BAND, steps=steps, batch=batch, seed=0)
        fit_s = time.perf_counter() - t
        sel = np.random.default_rng(0).choice(len(vals), nd, replace=False)
        t = time.perf_counter()
        F.decode_values(th, shapes, B, tr, (0, 0, 0), N_GRID, T.SDF, BAND, idx=sel)
        return steps * batch / fit_s, nd / (time.perf_counter() - t)

    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    fit_all, dec_all = rates(10, 1 << 20)
    with threadpool_limits(limits=1):
        fit_one, dec_one = rates(2, 1 << 15)
    extra = {}
    if moe_ctx is not None:
        from oracle import moe
        shapes_e = mlp.layer_shapes(K, W, H, C)
        ex = [dict(cell=c, theta=th_e.astype(np.float64), shapes=shapes_e, B=B, lo=lo_d[0], D=lo_d[1], scale=BAND)
              for c, (th_e, lo_d) in zip(moe_ctx["cells"], moe_ctx["experts"])]
        nm = 1 << 14
        sel_m = np.random.default_rng(1).choice(len(vals), nm, replace=False)
        t = time.perf_counter()
        moe.decode_moe(tr["ijk"][sel_m], ex, moe_ctx["origin"], moe_ctx["size"], moe_ctx["halo"])
        extra["moe_blend_voxels_per_s"] = nm / (time.perf_counter() - t)
    if c4_grads:
        extra["c4_gradient_check"] = c4_gradient_check(c4_grads)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {**extra, "value": fit_all, "unit": "train samples/s", "cores": int(threads), "kind": "oracle",
            "sample": "10 Adam steps x 2^14 samples of the 4x128 regressor on the same 512^3 volume, FP64 numpy on "
                      "all cores (oracle tree build of %d voxels took %.1f s, not counted); decode of 2^20 sampled "
                      "voxels for decode_voxels_per_s; single-thread rates from 2 steps x 2^14 and 2^15 decoded "
                      "voxels; blended decode (8 experts) of 2^14 sampled voxels for moe_blend_voxels_per_s"
                      % (len(vals), build_s),
            "decode_voxels_per_s": dec_all, "single_thread": {"train_samples_per_s": fit_one,
                                                              "decode_voxels_per_s": dec_one},
            "nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": _cpu_model()}


if __name__ == "__main__":
    main()
