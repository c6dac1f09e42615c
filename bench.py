"""Throughput benchmark of the sparse FastTucker SGD sweep on one MI355X.

A step is one SGD epoch over the whole training set: the factor epoch
(order, permutation, mode-sorted minibatch builder, per-minibatch
gather-contract-gradient and sorted segmented row updates) followed by the
core epoch (core-gradient partials and the fixed-order core update). The
metric is nonzeros per second per epoch = |Omega_train| / epoch time.

Default workload: the order-5 tensor 200,000 x 200,000 x 50,000 x 1,000 x 24
with 200M Zipf(1.1) nonzeros (180M train / 20M test) from a planted J = R = 32
model, minibatch 262,144, deterministic segmented reductions, per-row mean
steps. The headline runs the FP32 contraction; the same epochs are repeated
with the BF16 and the FP8 e4m3 contractions, with the contractions on vector
FMAs instead of the matrix cores, and (one epoch) in the Hogwild fast mode.

Every leg states its error against the FP64 oracle: on one full-size
minibatch from the leg's own parameters (loss, row gradients, occurrence
counts) and on the test SSE over a 1M-nonzero slice of the test set, both
computed by the oracle from the same parameters. Accuracy: test RMSE after
the workload's own epoch count from the common initial point, and its
relative difference from the FP32 leg (pass: within 1%).

Prints ONE JSON line on stdout; progress goes to stderr. Inputs are resident
in device memory before timing starts.
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
MFMA_PEAK_TFS = {"fp32": 157.3, "bf16": 2500.0, "fp8_e4m3": 5000.0}
FACTOR_KERNELS = ("factor_grad", "seg_reduce", "seg_combine")
TRAFFIC_SOURCES = ["paper_2404_10087_amd/csrc/k_factor.hip",
                   "paper_2404_10087_amd/csrc/mfma_tile.h",
                   "paper_2404_10087_amd/csrc/ft_internal.h"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------ method model
def factor_bytes_per_sample(N, sumJ):
    """Compulsory bytes of the factor phase per training nonzero with no
    cache reuse: int32 coordinates and the FP32 value (4N + 4), the gathered
    factor rows (4 sum J_n) and the updated rows written back (4 sum J_n)."""
    return 4 * N + 4 + 8 * sumJ


def core_bytes_per_sample(N, sumJ):
    """Core phase: coordinates, value and gathered rows (A is read-only)."""
    return 4 * N + 4 + 4 * sumJ


def factor_flops_per_sample(N, sumJ, R):
    """C = A_Psi B and g = r B d (2 R sum J_n each), the leave-one-out
    products 3 (N - 2) R, xhat 2R, and the row update 4 sum J_n."""
    return 4 * R * sumJ + 3 * (N - 2) * R + 2 * R + 4 * sumJ


def core_flops_per_sample(N, sumJ, R):
    """C = A_Psi B and Grad += E^T D (2 R sum J_n each), leave-one-out, xhat."""
    return 4 * R * sumJ + 3 * (N - 2) * R + 2 * R


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(workload_key):
    """HBM bytes per minibatch of the factor phase from the committed
    rocprofv3 counter summary, if it was taken on the current kernels."""
    path = os.path.join(ROOT, "profiles",
                        f"traffic_factor_phase_{workload_key}.txt")
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
        return float(rec["hbm_bytes_per_minibatch"])
    except (KeyError, ValueError):
        return None


# ------------------------------------------------------------ CPU baseline
def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(n, 1)


def cpu_baseline(w, T, A0, B0, mb_one, mb_all):
    """The FP64 oracle on the host: one factor epoch and one core epoch over
    the first training nonzeros (in stored order), once on one thread over
    mb_one minibatches and once on every allowed core over mb_all; scaled to
    nonzeros per second per epoch."""
    import oracle
    oracle.build()
    legs = {}
    for key, n_mb, threads, par in (("single_thread", mb_one, 1, False),
                                    ("all_cores", mb_all, host_threads(),
                                     True)):
        S = min(n_mb * w.M, T.train_idx.shape[1])
        used = oracle.set_threads(threads)
        idx = np.ascontiguousarray(T.train_idx[:, :S])
        val = T.train_val[:S].astype(np.float64)
        A = [a.astype(np.float64) for a in A0]
        B = [b.astype(np.float64) for b in B0]
        log(f"oracle {key}: {S} nonzeros on {used} thread(s)")
        t0 = time.perf_counter()
        oracle.factor_epoch(A, B, idx, val, np.arange(S), w.M, w.lr_A,
                            w.lam_A, w.row_mean, parallel=par)
        t1 = time.perf_counter()
        oracle.core_epoch(A, B, idx, val, w.lr_B, w.lam_B, parallel=par)
        t2 = time.perf_counter()
        legs[key] = {"value": S / (t2 - t0), "cores": used, "nnz": S,
                     "factor_s": round(t1 - t0, 3), "core_s": round(t2 - t1, 3)}
    oracle.set_threads(0)
    a = legs["all_cores"]
    return {"value": a["value"], "unit": "nonzeros/s", "cores": a["cores"],
            "kind": "oracle", "cpu": cpu_model(),
            "sample": (f"first {a['nnz']} training nonzeros "
                       f"({a['nnz'] // w.M} minibatches of {w.M}): one factor "
                       f"epoch ({a['factor_s']:.2f} s) and one core epoch "
                       f"({a['core_s']:.2f} s), FP64, {a['cores']} threads "
                       "(OpenMP over the samples of a minibatch, fixed-order "
                       "combination)"),
            "single_thread": legs["single_thread"]}


# ------------------------------------------------------------ oracle checks
def oracle_check(ft, w, T, test_slice):
    """The leg's GPU results against the FP64 oracle at the leg's current
    parameters: minibatch 0 of a freshly prepared epoch (sum r^2/2, the
    per-row gradient sums, the occurrence counts) and the test SSE over the
    first test_slice test nonzeros."""
    import oracle
    from paper_2404_10087_amd import FT_TEST
    oracle.set_threads(host_threads())
    A, B = ft.get_params()
    A64 = [a.astype(np.float64) for a in A]
    B64 = [b.astype(np.float64) for b in B]
    ft.prepare_epoch()
    gl, G, K = ft.factor_minibatch(0, apply=False)
    mb = ft.epoch_order()[:w.M]
    idx = np.ascontiguousarray(T.train_idx[:, mb])
    val = T.train_val[mb].astype(np.float64)
    ol, OG, OK = oracle.factor_minibatch(A64, B64, idx, val, 0.0, w.lam_A,
                                         w.row_mean, apply=False,
                                         want_grad=True, parallel=True)
    gerr = []
    for n in range(w.order):
        num = np.linalg.norm(G[n].astype(np.float64) - OG[n])
        den = np.linalg.norm(OG[n])
        gerr.append(float(num / den) if den > 0 else float(num))
    counts_equal = all(np.array_equal(K[n].astype(np.int64), OK[n])
                       for n in range(w.order))
    S = min(test_slice, T.test_idx.shape[1])
    tidx = np.ascontiguousarray(T.test_idx[:, :S])
    tval = T.test_val[:S]
    ft.set_nonzeros(FT_TEST, tidx, tval)
    gsse, _ = ft.eval(FT_TEST)
    osse, _ = oracle.residual_stats(A64, B64, tidx, tval.astype(np.float64),
                                    parallel=True)
    ft.set_nonzeros(FT_TEST, T.test_idx, T.test_val)
    return {"minibatch_samples": int(len(mb)),
            "minibatch_loss_rel_err": abs(gl - ol) / abs(ol),
            "row_grad_rel_err_max_mode": max(gerr),
            "row_grad_rel_err_per_mode": [float(f"{e:.3e}") for e in gerr],
            "occurrence_counts_equal": bool(counts_equal),
            "test_slice_nonzeros": int(S),
            "test_sse_rel_err": abs(gsse - osse) / abs(osse)}


# ------------------------------------------------------------ legs
def run_leg(name, w, T, A0, B0, args, precision, options):
    from paper_2404_10087_amd import (FT_ROW_MEAN, FT_ROW_SUM, FT_TEST,
                                      FT_TRAIN, FastTucker, FtError)
    ft = FastTucker(w.dims, w.J, w.R)
    try:
        ft.set_options(minibatch=w.M, lr_A=w.lr_A, lr_B=w.lr_B,
                       lambda_A=w.lam_A, lambda_B=w.lam_B,
                       row_scale=FT_ROW_MEAN if w.row_mean else FT_ROW_SUM,
                       shuffle_seed=w.order_seed, reshuffle_each_epoch=1,
                       precision=precision, **options)
        ft.set_nonzeros(FT_TRAIN, T.train_idx, T.train_val)
        ft.set_nonzeros(FT_TEST, T.test_idx, T.test_val)
        nnz = T.train_idx.shape[1]
        hog = options.get("deterministic", 1) == 0
        out = {}
        # accuracy: the workload's epoch count from the common initial point
        acc_epochs = 0 if hog or args.no_accuracy else w.epochs
        ft.set_params(A0, B0)
        curve = [ft.rmse(FT_TEST)]
        for e in range(acc_epochs):
            ft.epoch_factors()
            ft.epoch_core()
            curve.append(ft.rmse(FT_TEST))
        if acc_epochs:
            out["test_rmse_after_epochs"] = acc_epochs
            out["test_rmse"] = curve[-1]
            out["test_rmse_curve"] = [round(v, 6) for v in curve]
            log(f"{name}: test RMSE {curve[0]:.5f} -> {curve[-1]:.5f} after "
                f"{acc_epochs} epochs")
        # throughput: warmup, then exactly the timed epochs, from the
        # initial point again
        ft.set_params(A0, B0)
        warm = 0 if hog else args.warmup
        steps = args.hogwild_steps if hog else args.steps
        for _ in range(warm):
            ft.epoch_factors()
            ft.epoch_core()
        t_f = t_c = 0.0
        t0 = time.perf_counter()
        for _ in range(steps):
            a = time.perf_counter()
            ft.epoch_factors()
            b = time.perf_counter()
            ft.epoch_core()
            c = time.perf_counter()
            t_f += b - a
            t_c += c - b
        el = time.perf_counter() - t0
        out.update({"value": nnz / (el / steps), "steps": steps,
                    "warmup": warm, "ms_per_step": 1000.0 * el / steps,
                    "factor_nnz_per_s": nnz / (t_f / steps),
                    "core_nnz_per_s": nnz / (t_c / steps),
                    "phase_ms_per_epoch": {"factor": 1000 * t_f / steps,
                                           "core": 1000 * t_c / steps}})
        log(f"{name}: {out['value']:.4g} nonzeros/s ({out['ms_per_step']:.2f}"
            f" ms per epoch over {steps} epochs)")
        if hog:
            out["test_rmse_after_timed_epochs"] = ft.rmse(FT_TEST)
        # per-kernel device time from HIP events over further epochs
        ft.profile(True)
        ft.profile_reset()
        for _ in range(1 if hog else args.profile_steps):
            ft.epoch_factors()
            ft.epoch_core()
        from paper_2404_10087_amd import KERNELS
        stats = {k: ft.profile_get(k) for k in KERNELS}
        ft.profile(False)
        out["kernels"] = {k: {"launches": v[0], "total_ms": round(v[1], 4),
                              "avg_us": round(1000 * v[1] / v[0], 3)}
                          for k, v in stats.items() if v[0]}
        out["profiled_epochs"] = 1 if hog else args.profile_steps
        if not hog:
            # the builder alone (in line on the library stream, full grids):
            # during the timed epochs it runs beside the core phase, where
            # its event times include the sharing
            ft.prepare_epoch()
            a = time.perf_counter()
            for _ in range(2):
                ft.prepare_epoch()
            out["builder_alone_ms"] = 1000.0 * (time.perf_counter() - a) / 2
        if not hog and not args.no_oracle_check:
            log(f"{name}: oracle check")
            out["oracle_check"] = oracle_check(ft, w, T, args.test_slice)
        return out
    except FtError as e:
        log(f"{name}: {e}")
        return {"error": str(e)}
    finally:
        ft.close()


def roofline(w, leg, n_mb, nnz):
    """Method bytes of the factor phase per minibatch (factor_grad +
    seg_reduce + seg_combine) over its mean duration from HIP events, and
    the same for the core phase per epoch."""
    k = leg["kernels"]
    epochs = leg["profiled_epochs"]
    sumJ = w.J * w.order
    m = nnz / n_mb
    t_fac = sum(k[x]["total_ms"] for x in FACTOR_KERNELS if x in k) / 1000.0
    t_mb = t_fac / (epochs * n_mb)
    fb = factor_bytes_per_sample(w.order, sumJ) * m
    ach = fb / t_mb / 1e9
    t_core = k["core_grad"]["total_ms"] / 1000.0 / epochs
    cb = core_bytes_per_sample(w.order, sumJ) * nnz
    return {"fac_bytes": fb, "fac_s": t_mb, "fac_gbs": ach,
            "fac_tfs": factor_flops_per_sample(w.order, sumJ, w.R) * m /
            t_mb / 1e12,
            "core_bytes": cb, "core_s": t_core, "core_gbs": cb / t_core / 1e9,
            "core_tfs": core_flops_per_sample(w.order, sumJ, w.R) * nnz /
            t_core / 1e12}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="epochs after the timed ones with kernel events on")
    ap.add_argument("--config", default="c3")
    ap.add_argument("--legs", default="fp32,bf16,fp8_e4m3,fp32_vector_alu,"
                    "fp32_core_storage,hogwild_fp32")
    ap.add_argument("--hogwild-steps", type=int, default=1)
    ap.add_argument("--cpu-minibatches", type=int, default=1,
                    help="minibatches of the 1-thread oracle leg")
    ap.add_argument("--cpu-minibatches-all", type=int, default=16,
                    help="minibatches of the all-core oracle leg")
    ap.add_argument("--test-slice", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the accuracy epochs (profiling runs)")
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
        print(f"bench.py measures one GPU only (asked for {args.gpus}): this "
              "build has no multi-GPU path; how it would shard is described "
              "in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import synth

    w = synth.get(args.config)
    t_gen = time.perf_counter()
    T = synth.make_tensor(w, cache_dir=args.cache_dir, progress=log)
    A0, B0 = synth.init_params(w.init_seed, w.dims, w.J, w.R, w.init_a_std,
                               w.init_b_std, w.init_dist)
    t_gen = time.perf_counter() - t_gen
    nnz = T.train_idx.shape[1]
    n_mb = (nnz + w.M - 1) // w.M
    log(f"generated {w.name}: {nnz} train / {T.test_idx.shape[1]} test "
        f"nonzeros in {t_gen:.1f} s")

    leg_defs = {"fp32": (0, {}), "bf16": (1, {}), "fp8_e4m3": (2, {}),
                "fp32_vector_alu": (0, {"vector_alu": 1}),
                "fp32_core_storage": (0, {"core_storage": 1}),
                "hogwild_fp32": (0, {"deterministic": 0})}
    names = [x for x in args.legs.split(",") if x]
    if "fp32" not in names:
        names.insert(0, "fp32")
    legs = {}
    for name in names:
        prec, opts = leg_defs[name]
        legs[name] = run_leg(name, w, T, A0, B0, args, prec, opts)
    head = legs["fp32"]
    if "error" in head:
        raise SystemExit(f"FP32 leg failed: {head['error']}")
    if "test_rmse" not in head:
        head["test_rmse"] = None

    # accuracy of every leg against the FP32 leg (same initial point and
    # epoch count)
    for name, leg in legs.items():
        if name == "fp32" or "test_rmse" not in leg or \
                head["test_rmse"] is None:
            continue
        rel = leg["test_rmse"] / head["test_rmse"] - 1.0
        leg["test_rmse_rel_to_fp32"] = rel
        leg["within_1pct_of_fp32"] = abs(rel) <= 0.01

    # rooflines from the FP32 leg (and per low-precision leg)
    rf = roofline(w, head, n_mb, nnz)
    for name in ("bf16", "fp8_e4m3", "fp32_vector_alu", "fp32_core_storage"):
        if name in legs and "kernels" in legs[name]:
            r = roofline(w, legs[name], n_mb, nnz)
            dt = "fp32" if name.startswith("fp32") else name
            legs[name]["roofline"] = {
                "factor_phase_gbs": r["fac_gbs"],
                "factor_phase_hbm_frac": r["fac_gbs"] / HBM_PEAK_GBS,
                "factor_phase_tflops": r["fac_tfs"],
                "core_phase_gbs": r["core_gbs"],
                "core_phase_tflops": r["core_tfs"],
                "mfma_peak_tflops": MFMA_PEAK_TFS[dt]}
    traffic = read_traffic(args.config)
    kf = head["kernels"]
    avg_us = {x: kf[x]["avg_us"] for x in FACTOR_KERNELS if x in kf}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, T, A0, B0, args.cpu_minibatches,
                           args.cpu_minibatches_all)

    sumJ = w.J * w.order
    line = {
        "metric": METRIC, "value": head["value"], "unit": "nonzeros/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "order": w.order,
                   "dims": list(w.dims), "nnz_train": nnz,
                   "nnz_test": int(T.test_idx.shape[1]), "J": w.J, "R": w.R,
                   "minibatch": w.M, "minibatches": n_mb,
                   "precision": "fp32", "lr_A": w.lr_A, "lr_B": w.lr_B,
                   "lambda": w.lam_A,
                   "row_scale": "mean" if w.row_mean else "sum",
                   "core_step": "per_epoch", "deterministic": True,
                   "reshuffle_each_epoch": True, "epochs": w.epochs},
        "roofline": {
            "bound": "hbm",
            "kernel": "factor phase per minibatch: factor_grad + seg_reduce"
                      " (+ seg_combine)",
            "achieved": rf["fac_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": rf["fac_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
            "alg_bytes_per_launch": rf["fac_bytes"],
            "alg_bytes_per_sample": factor_bytes_per_sample(w.order, sumJ),
            "avg_launch_us": rf["fac_s"] * 1e6,
            "avg_kernel_us": avg_us,
            "timing": "HIP events on the library stream over "
                      f"{args.profile_steps} epochs after the timed ones",
            "mfma": {"achieved_tflops": rf["fac_tfs"],
                     "peak_tflops": MFMA_PEAK_TFS["fp32"],
                     "frac": rf["fac_tfs"] / MFMA_PEAK_TFS["fp32"],
                     "flops_per_sample":
                         factor_flops_per_sample(w.order, sumJ, w.R)},
            "core_phase": {
                "kernel": "core_grad per epoch",
                "achieved_gbs": rf["core_gbs"],
                "frac": rf["core_gbs"] / HBM_PEAK_GBS,
                "alg_bytes_per_sample": core_bytes_per_sample(w.order, sumJ),
                "avg_launch_us": rf["core_s"] * 1e6,
                "mfma_tflops": rf["core_tfs"],
                "mfma_frac": rf["core_tfs"] / MFMA_PEAK_TFS["fp32"]}},
        "cpu_baseline": cpu,
        "phase_ms_per_epoch": head["phase_ms_per_epoch"],
        "factor_nnz_per_s": head["factor_nnz_per_s"],
        "core_nnz_per_s": head["core_nnz_per_s"],
        "builder_kernel_ms_per_epoch": sum(
            kf[x]["total_ms"] for x in ("order", "permute", "sort")
            if x in kf) / head["profiled_epochs"],
        "builder_alone_ms_per_epoch": head.get("builder_alone_ms"),
        "test_rmse": head.get("test_rmse"),
        "test_rmse_after_epochs": head.get("test_rmse_after_epochs"),
        "oracle_check": head.get("oracle_check"),
        "legs": {k: v for k, v in legs.items() if k != "fp32"},
        "kernels": kf,
        "generation_s": round(t_gen, 1),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
