"""Throughput benchmark of the sparse FastTucker SGD sweep on one MI355X.

A step is one SGD epoch over the whole training set: the factor epoch
(order, permutation, mode-sorted minibatch builder, per-minibatch
gather-contract-gradient and sorted segmented row updates) followed by the
core epoch (core-gradient partials and the fixed-order core update). The
metric is nonzeros per second per epoch = |Omega_train| / epoch time.

Workload (default): the order-3 rating-shaped tensor 20,000 x 20,000 x 1,000
with 10M Zipf(1.1) nonzeros (9M train / 1M test), J = R = 16, minibatch
65,536, FP32, deterministic segmented reductions, per-row mean steps.

Prints ONE JSON line. Inputs are resident in device memory before timing.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("nonzeros/sec per SGD epoch (factor+core) at 1 GPU, FP32 vs "
          "BF16/FP8 at test RMSE")
HBM_PEAK_GBS = 8000.0
DOMINANT = "factor_grad"


def algorithmic_bytes_per_sample(kernel, N, J, J4):
    """Compulsory bytes one sample moves in a kernel (no cache reuse):
    int32 coordinates and the FP32 value, the gathered factor rows (J_n
    floats each), and for the factor kernel the per-sample row gradients it
    writes (J4 floats per mode)."""
    stream = 4 * N + 4
    rows = 4 * J * N
    if kernel == "factor_grad":
        return stream + rows + 4 * J4 * N
    if kernel in ("core_grad", "eval"):
        return stream + rows
    raise KeyError(kernel)


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


TRAFFIC_SOURCES = ["paper_2404_10087_amd/csrc/k_factor.hip",
                   "paper_2404_10087_amd/csrc/mfma_tile.h"]


def read_traffic(workload):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{DOMINANT}_{workload}.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("source_digest") != source_digest(TRAFFIC_SOURCES):
        return None
    try:
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, T, A0, B0, sample_nnz):
    """The FP64 oracle, single thread, on the first sample_nnz training
    nonzeros of the epoch-0 order: one factor epoch and one core epoch over
    that subset; scaled to nonzeros/s per epoch."""
    import oracle
    oracle.build()
    perm = np.arange(T.train_idx.shape[1])[:sample_nnz]
    idx = np.ascontiguousarray(T.train_idx[:, perm])
    val = T.train_val[perm].astype(np.float64)
    A = [a.astype(np.float64) for a in A0]
    B = [b.astype(np.float64) for b in B0]
    t0 = time.perf_counter()
    oracle.factor_epoch(A, B, idx, val, np.arange(sample_nnz), w.M, w.lr_A,
                        w.lam_A, w.row_mean)
    t1 = time.perf_counter()
    oracle.core_epoch(A, B, idx, val, w.lr_B, w.lam_B)
    t2 = time.perf_counter()
    return {"value": sample_nnz / (t2 - t0), "unit": "nonzeros/s",
            "cores": 1, "kind": "oracle",
            "sample": (f"first {sample_nnz} training nonzeros "
                       f"({sample_nnz // w.M} minibatches of {w.M}): one "
                       f"factor epoch ({t1 - t0:.2f} s) and one core epoch "
                       f"({t2 - t1:.2f} s), FP64, 1 thread")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="epochs after the timed ones with kernel events on")
    ap.add_argument("--config", default="c1")
    ap.add_argument("--cpu-sample", type=int, default=46 * 65536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-low-precision", action="store_true",
                    help="skip the BF16, FP8, Hogwild and vector-ALU "
                    "comparison runs")
    ap.add_argument("--cache-dir", default=os.environ.get("FT_SYNTH_CACHE"),
                    help="reuse the generated tensor across runs")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    metavar="MiB", help="only run a plain device copy of this "
                    "many MiB (known traffic for scaling HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n,
                          "copy_calibration_bytes_written": 4 * n}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the "
              "multi-GPU design is described but not built", file=sys.stderr)
        sys.exit(2)

    import synth
    from paper_2404_10087_amd import (FT_ROW_MEAN, FT_ROW_SUM, FT_TEST,
                                      FT_TRAIN, FastTucker, FtError)

    w = synth.get(args.config)
    t_gen = time.perf_counter()
    T = synth.make_tensor(
        w, cache_dir=args.cache_dir,
        progress=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
    A0, B0 = synth.init_params(w.init_seed, w.dims, w.J, w.R, w.init_a_std,
                               w.init_b_std, w.init_dist)
    t_gen = time.perf_counter() - t_gen
    nnz = T.train_idx.shape[1]
    print(f"[bench] generated {w.name}: {nnz} train / "
          f"{T.test_idx.shape[1]} test nonzeros in {t_gen:.1f} s",
          file=sys.stderr, flush=True)

    def make(precision):
        ft = FastTucker(w.dims, w.J, w.R)
        ft.set_options(minibatch=w.M, lr_A=w.lr_A, lr_B=w.lr_B,
                       lambda_A=w.lam_A, lambda_B=w.lam_B,
                       row_scale=FT_ROW_MEAN if w.row_mean else FT_ROW_SUM,
                       shuffle_seed=w.order_seed, reshuffle_each_epoch=1,
                       precision=precision)
        ft.set_nonzeros(FT_TRAIN, T.train_idx, T.train_val)
        ft.set_nonzeros(FT_TEST, T.test_idx, T.test_val)
        ft.set_params(A0, B0)
        return ft

    def timed(ft):
        """warmup, then exactly args.steps epochs (factor + core); kernel
        events off, every epoch call returns synchronised."""
        for _ in range(args.warmup):
            ft.epoch_factors()
            ft.epoch_core()
        t_f = t_c = 0.0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            a = time.perf_counter()
            ft.epoch_factors()
            b = time.perf_counter()
            ft.epoch_core()
            c = time.perf_counter()
            t_f += b - a
            t_c += c - b
        return time.perf_counter() - t0, t_f, t_c

    ft = make(0)
    rmse0 = ft.rmse(FT_TEST)
    elapsed, t_factor, t_core = timed(ft)
    # per-kernel durations from HIP events on the library's stream, over
    # further epochs of the same run
    ft.profile(True)
    ft.profile_reset()
    for _ in range(args.profile_steps):
        ft.epoch_factors()
        ft.epoch_core()
    stats = {k: ft.profile_get(k) for k in
             ("order", "permute", "sort", "factor_grad", "seg_reduce",
              "core_grad", "core_update")}
    ft.profile(False)
    rmse = ft.rmse(FT_TEST)
    train_rmse = ft.rmse(FT_TRAIN)
    ms_per_step = 1000.0 * elapsed / args.steps
    value = nnz / (elapsed / args.steps)

    # roofline of the dominant kernel: algorithmic bytes / mean launch time
    n_launch, tot_ms = stats[DOMINANT]
    J4 = (w.J + 3) // 4 * 4
    samples_per_launch = nnz / ft.num_minibatches()
    alg_bytes = algorithmic_bytes_per_sample(DOMINANT, w.order, w.J, J4) * \
        samples_per_launch
    avg_s = tot_ms / 1000.0 / max(n_launch, 1)
    achieved = alg_bytes / avg_s / 1e9
    traffic = read_traffic(args.config)
    kernel_ms = {k: {"launches": v[0], "total_ms": round(v[1], 4),
                     "avg_us": round(1000 * v[1] / max(v[0], 1), 3)}
                 for k, v in stats.items()}

    # the same epochs with the low-precision contractions, with the Hogwild
    # fast mode and with vector-ALU factor contractions (same initial
    # parameters and epoch orders), each with its own test RMSE
    low = {}
    for pname, pcode in (("bf16", 1), ("fp8_e4m3", 2), ("hogwild_fp32", 0),
                         ("fp32_vector_alu", 0)):
        if args.no_low_precision:
            break
        del ft
        ft = make(pcode)
        try:
            if pname.startswith("hogwild"):
                # the paper's execution model: no minibatch barrier, atomic
                # per-tile row updates (not reproducible; for comparison)
                ft.set_options(deterministic=0)
            if pname.endswith("vector_alu"):
                # matrix-core ablation: factor contractions on vector FMAs
                ft.set_options(vector_alu=1)
        except FtError as e:
            low[pname] = {"error": str(e)}
            continue
        try:
            el, tf, tc = timed(ft)
            ft.profile(True)     # same epoch count as FP32, kernel events on
            ft.profile_reset()
            for _ in range(args.profile_steps):
                ft.epoch_factors()
                ft.epoch_core()
            lstats = {k: ft.profile_get(k) for k in
                      ("factor_grad", "seg_reduce", "hogwild",
                       "core_grad")}
            ft.profile(False)
        except FtError as e:     # e.g. a Hogwild run that diverges
            low[pname] = {"error": str(e)}
            continue
        low[pname] = {"value": nnz / (el / args.steps),
                      "ms_per_step": 1000.0 * el / args.steps,
                      "factor_nnz_per_s": nnz / (tf / args.steps),
                      "core_nnz_per_s": nnz / (tc / args.steps),
                      "test_rmse": ft.rmse(FT_TEST),
                      "kernel_avg_us": {
                          k: round(1000 * v[1] / max(v[0], 1), 3)
                          for k, v in lstats.items() if v[0]}}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, T, A0, B0, min(args.cpu_sample, nnz))

    line = {
        "metric": METRIC, "value": value, "unit": "nonzeros/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "order": w.order,
                   "dims": list(w.dims), "nnz_train": nnz,
                   "nnz_test": int(T.test_idx.shape[1]), "J": w.J, "R": w.R,
                   "minibatch": w.M, "precision": "fp32",
                   "row_scale": "mean" if w.row_mean else "sum",
                   "core_step": "per_epoch", "deterministic": True,
                   "reshuffle_each_epoch": True},
        "roofline": {"bound": "hbm", "kernel": DOMINANT,
                     "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes,
                     "timing": "HIP events on the library stream over "
                               f"{args.profile_steps} epochs after the timed "
                               "ones (events inside the timed epochs slow "
                               "them)",
                     "avg_launch_us": avg_s * 1e6},
        "cpu_baseline": cpu,
        "phase_ms_per_epoch": {"factor": 1000 * t_factor / args.steps,
                               "core": 1000 * t_core / args.steps},
        "factor_nnz_per_s": nnz / (t_factor / args.steps),
        "core_nnz_per_s": nnz / (t_core / args.steps),
        "builder_ms_per_epoch": sum(stats[k][1] for k in
                                    ("order", "permute", "sort"))
        / max(stats["sort"][0], 1),
        "low_precision": low,
        "kernels": kernel_ms,
        "test_rmse": rmse, "train_rmse": train_rmse,
        "test_rmse_initial": rmse0,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
