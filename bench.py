"""Benchmark of the GP hot path on one MI355X.

One step is one pass of the whole path over the n=65536, D=128 workload (8192 test
points, tile 2048), in float64 and in the mixed precisions (FP32 trailing updates and the
3-way split-bfloat16 products with six and with three products by default): covariance
assembly, tiled Cholesky, alpha (with the precision's default float64 refinement sweeps in
the mixed modes), NLML, posterior mean, posterior variance and the NLML gradient.  Inputs
are resident in HBM before the timed region; every phase is timed with HIP events on the
stream the library launches on.

Prints one JSON line.  ``value`` is the float64 Cholesky rate, (n^3/3 + n^2/2 + n/6)
flops divided by the median time of gpr_cholesky over the timed steps (each phase also
gets its median and mean with 95 % confidence intervals).  ``roofline`` covers the
dominant kernel of the float64 path (the timed tile-GEMM kernel with the most time over
the timed steps: the Cholesky trailing update, the inversion steps or the K^-1 trace
products of the gradient), from the library's event hook: algorithmic flops per launch /
average launch duration; ``kernels`` lists the same figures for every timed kernel.
``cpu_baseline`` is the FP64 CPU oracle's train step and prediction timed on the host on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Cholesky TFLOP/s + train/predict s, n=65536 D=128: FP64 vs mixed @ stated err"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
SPLIT_PRODUCTS = {"bf16x3": 3, "bf16x6": 6, "bf16x3_trtri": 3, "bf16x6_trtri": 6, "bf16x3_trace": 3, "bf16x6_trace": 6}
WORKLOADS = {
    # the configuration the metric is quoted on: n=65536, D=128 lagged inputs, 8192 test points, tile 2048
    "n65536_d128": dict(n=65536, m=8192, D=128, tile=2048, seed=3),
    # smaller shapes of the same generator (for quick runs)
    "n16384_d8": dict(n=16384, m=4096, D=8, tile=1024, seed=2),
    "n4096_d128": dict(n=4096, m=1024, D=128, tile=1024, seed=3),
}


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "gemm_kernel_traffic.json")
# the sources of each tile-product kernel family; a traffic figure is reported only while
# its family's sources are the ones it was measured with
KERNEL_SOURCES = {"f64_f32": [os.path.join(ROOT, "paper_2505_00136_amd", "csrc", f) for f in ("gemm.hip", "gemm_device.h")],
                  "bf16": [os.path.join(ROOT, "paper_2505_00136_amd", "csrc", "gemm_bf16.hip")]}


def kernel_family(kernel: str) -> str:
    return "bf16" if "bf16" in kernel else "f64_f32"
# timing kinds of the library's event hook -> kernel symbol, operand dtype.  The symbols are
# the operand-mode specialisations that run for this workload's whole 2048-wide tiles
# (update and trace: MC/MC = 3; the inversion's row-scaling launches are KC/MC = 1 and its
# elimination launches MC/MC = 3, and the hook times both, hence `*`; the split-bf16 update
# runs its 256 x 256 macro-tile kernel, as tile edges that are multiples of 256 do).
TIMED_KERNELS = {
    "fp64": ("gemm_update_kernel<double, 3>", "f64"), "fp32": ("gemm_update_kernel<float, 3>", "f32"),
    "fp64_trtri": ("gemm_trtri_kernel<double, *>", "f64"), "fp32_trtri": ("gemm_trtri_kernel<float, *>", "f32"),
    "fp64_trace": ("gemm_trace_kernel<double, 3>", "f64"), "fp32_trace": ("gemm_trace_kernel<float, 3>", "f32"),
    "bf16x3": ("gemm_bf16x_t256_kernel<3>", "bf16"), "bf16x6": ("gemm_bf16x_t256_kernel<6>", "bf16"),
    "bf16x3_trtri": ("gemm_bf16x_trtri_t256_kernel<3>", "bf16"), "bf16x6_trtri": ("gemm_bf16x_trtri_t256_kernel<6>", "bf16"),
    "bf16x3_trace": ("gemm_bf16x_trace_t256_kernel<3>", "bf16"), "bf16x6_trace": ("gemm_bf16x_trace_t256_kernel<6>", "bf16"),
}
KIND_ROLE = {"fp64": "trailing SYRK+GEMM update of a Cholesky step", "fp32": "trailing SYRK+GEMM update of a Cholesky step",
             "fp64_trtri": "step of the triangular inversion L^-1 (gradient)",
             "fp32_trtri": "step of the triangular inversion L^-1 (gradient)",
             "fp64_trace": "K^-1 block-row product fused with the gradient reduction",
             "fp32_trace": "K^-1 block-row product fused with the gradient reduction",
             "bf16x3": "trailing update of a Cholesky step from split-bf16 planes",
             "bf16x6": "trailing update of a Cholesky step from split-bf16 planes",
             "bf16x3_trtri": "step of the triangular inversion L^-1 (gradient) from split-bf16 planes",
             "bf16x6_trtri": "step of the triangular inversion L^-1 (gradient) from split-bf16 planes",
             "bf16x3_trace": "K^-1 block-row product fused with the gradient reduction, split-bf16 planes",
             "bf16x6_trace": "K^-1 block-row product fused with the gradient reduction, split-bf16 planes"}


def source_digest(paths) -> str:
    """First 16 hex digits of the sha256 of the concatenated kernel sources."""
    import hashlib
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter record, or None when the
    record is missing, does not cover the kernel, or the kernel's sources changed since."""
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    fam = kernel_family(kernel)
    if rec.get("source_families", {}).get(fam, {}).get("sha256_16") != source_digest(KERNEL_SOURCES[fam]):
        return None
    return rec.get("bytes_per_launch", {}).get(kernel)


def copy_calibration(nbytes: int):
    """A plain device-to-device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes}))


def chol_flops(n: int) -> float:
    return n ** 3 / 3.0 + n ** 2 / 2.0 + n / 6.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def spread(xs):
    """Median and mean of repeated timings with 95 % confidence intervals: the median's from
    order statistics (the widest pair of ranks whose binomial(K, 1/2) coverage is >= 95 %;
    min and max when K is too small for that), the mean's from Student's t."""
    from scipy import stats as st
    x = np.sort(np.asarray(xs, dtype=np.float64))
    k = x.size
    out = {"runs": int(k), "median": float(np.median(x)), "mean": float(np.mean(x))}
    j = 0
    while j + 1 <= k // 2 and st.binom.cdf(j, k, 0.5) <= 0.025:
        j += 1
    out["ci95_median"] = [float(x[j - 1]), float(x[k - j])] if j >= 1 else [float(x[0]), float(x[-1])]
    out["ci95_median_coverage"] = float(1 - 2 * st.binom.cdf(j - 1, k, 0.5)) if j >= 1 else None
    if k > 1:
        half = float(st.t.ppf(0.975, k - 1) * np.std(x, ddof=1) / math.sqrt(k))
        out["ci95_mean"] = [out["mean"] - half, out["mean"] + half]
    return out


def host_blas():
    """BLAS libraries numpy/scipy use on this host, with their thread counts."""
    try:
        import threadpoolctl
        return [{"vendor": i.get("internal_api"), "version": i.get("version"), "threads": i.get("num_threads"),
                 "arch": i.get("architecture"), "lib": os.path.basename(i.get("filepath", ""))}
                for i in threadpoolctl.threadpool_info() if i.get("user_api") == "blas"]
    except Exception:
        return []


def cpu_baseline(wl, n_s=2048, m_s=512, runs=7):
    """The oracle's train step (assemble, Cholesky, alpha, NLML, gradient) and prediction
    (mean, variance) on the leading points of the same workload, timed on the host's cores
    (seven runs, median and 95 % CI per phase; about 10-30 s of host work); value = its
    Cholesky rate."""
    import datagen
    import oracle
    blas = host_blas()
    threads = max([b["threads"] or 1 for b in blas] or [os.cpu_count() or 1])
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=n_s, n_test=m_s, D=wl["D"], seed=wl["seed"]))
    h = oracle.Hyper(math.sqrt(wl["D"]), 1.0, 0.01)
    a = np.random.default_rng(0).normal(size=(2048, 2048))
    t0 = time.perf_counter()
    a @ a
    gemm_tflops = 2 * 2048 ** 3 / (time.perf_counter() - t0) / 1e12
    phases = {k: [] for k in ("assemble", "cholesky", "solve", "nlml", "grad", "mean", "var")}
    for _ in range(runs):
        t = [time.perf_counter()]
        K = oracle.train_cov(ds.Z, h)
        t.append(time.perf_counter())
        L = oracle.cholesky(K)
        t.append(time.perf_counter())
        al = oracle.solve_alpha(L, ds.y)
        t.append(time.perf_counter())
        oracle.nlml(L, ds.y, al)
        t.append(time.perf_counter())
        oracle.nlml_grad(ds.Z, h, L, al)
        t.append(time.perf_counter())
        oracle.predict_mean(ds.Z, ds.Zs, h, al)
        t.append(time.perf_counter())
        oracle.predict_var(ds.Z, ds.Zs, h, L)
        t.append(time.perf_counter())
        for k, (t0_, t1_) in zip(phases, zip(t[:-1], t[1:])):
            phases[k].append(t1_ - t0_)
    ph = {k: spread(v) for k, v in phases.items()}
    train = [sum(phases[k][r] for k in ("assemble", "cholesky", "solve", "nlml", "grad")) for r in range(runs)]
    pred = [phases["mean"][r] + phases["var"][r] for r in range(runs)]
    t_c = ph["cholesky"]["median"]
    return {"value": chol_flops(n_s) / t_c / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle (numpy/scipy float64, LAPACK dpotrf) train step and prediction on the first {n_s} "
                      f"training and {m_s} test points of the same workload (D={wl['D']}, same hyperparameters), "
                      f"{runs} runs; value = its Cholesky rate at the median time",
            "os_cpu_count": os.cpu_count(), "blas": blas, "host_dgemm_2048_tflops": round(gemm_tflops, 4),
            "train_step_s": spread(train), "predict_s": spread(pred), "phases_s": ph}


class Phases:
    def __init__(self, torch, stream):
        self.torch = torch
        self.stream = stream
        self.marks = []

    def mark(self, name):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        self.marks.append((name, e))

    def durations(self):
        out = {}
        for (n0, e0), (n1, e1) in zip(self.marks[:-1], self.marks[1:]):
            out[n1] = out.get(n1, 0.0) + e0.elapsed_time(e1) / 1e3
        return out


def run(args):
    import torch
    from paper_2505_00136_amd import _lib
    import datagen

    wl = WORKLOADS[args.workload]
    n, m, D, tile = wl["n"], wl["m"], wl["D"], wl["tile"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    log(f"[bench] workload {args.workload}: n={n} m={m} D={D} tile={tile}; generating data")
    ds = datagen.make_dataset(datagen.MSDConfig(n_train=n, n_test=m, D=D, seed=wl["seed"]))
    # hyperparameters: unit signal variance, noise 0.01, lengthscale sqrt(D) so that K is dense
    h = (math.sqrt(D), 1.0, 0.01, args.kernel)
    Z = torch.tensor(ds.Z, device=dev)
    Zs = torch.tensor(ds.Zs, device=dev)
    y = torch.tensor(ds.y, device=dev)
    precs = args.precs.split(",")
    Ks = {p: torch.empty(_lib.gpr_tiles_bytes(n, tile, p), dtype=torch.uint8, device=dev) for p in precs}
    wsb = max(_lib.gpr_workspace_size(n, m, D, tile, p) for p in precs)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    for p in precs:
        _lib.gpr_init(n, m, tile, p)   # the library's streams, events and staging ring, outside the timed steps
    outs = {p: dict(alpha=torch.empty(n, dtype=torch.float64, device=dev),
                    nlml=torch.empty(1, dtype=torch.float64, device=dev),
                    mean=torch.empty(m, dtype=torch.float64, device=dev),
                    var=torch.empty(m, dtype=torch.float64, device=dev),
                    grad=torch.empty(3, dtype=torch.float64, device=dev)) for p in precs}
    torch.cuda.synchronize()
    log(f"[bench] allocated {sum(k.numel() for k in Ks.values()) / 2**30:.1f} GiB tiles + {wsb / 2**30:.1f} GiB workspace")

    def one_step(ph: Phases):
        for p in precs:
            o = outs[p]
            K = Ks[p]
            sweeps = -1   # the library's default for the precision (0 in float64)
            ph.mark(f"{p}:start")
            _lib.gpr_assemble(Z, n, D, h, tile, p, K)
            ph.mark(f"{p}:assemble")
            _lib.gpr_cholesky(K, n, tile, p, ws, wsb, want_info=False)
            ph.mark(f"{p}:cholesky")
            if p == "fp64" and args.device_schedule:
                # the same factorisation once more, scheduled by the task graph on the device
                _lib.gpr_assemble(Z, n, D, h, tile, p, K)
                ph.mark(f"{p}:assemble_again")
                _lib.gpr_set_schedule("device")
                _lib.gpr_cholesky(K, n, tile, p, ws, wsb, want_info=False)
                _lib.gpr_set_schedule("lookahead")
                ph.mark(f"{p}:cholesky_device")
            _lib.gpr_solve(K, Z, n, D, h, tile, p, y, o["alpha"], sweeps, ws, wsb)
            ph.mark(f"{p}:solve")
            _lib.gpr_nlml(K, n, tile, p, y, o["alpha"], o["nlml"])
            ph.mark(f"{p}:nlml")
            _lib.gpr_predict(Z, n, Zs, m, D, h, o["alpha"], o["mean"], ws, wsb)
            ph.mark(f"{p}:mean")
            _lib.gpr_predict_var(Z, n, Zs, m, D, h, K, tile, p, False, False, o["var"], ws, wsb)
            ph.mark(f"{p}:var")
            _lib.gpr_nlml_grad(Z, n, D, h, K, tile, p, o["alpha"], (1, 1, 1), o["grad"], ws, wsb)
            ph.mark(f"{p}:grad")

    for w in range(args.warmup):
        log(f"[bench] warmup step {w + 1}/{args.warmup}")
        one_step(Phases(torch, stream))
        torch.cuda.synchronize()
    for p in _lib.TIMING_KINDS:
        _lib.gpr_timing_read(p)     # drop anything recorded so far
    _lib.gpr_timing_enable(True)
    per_step = {}   # phase -> durations of the timed steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ph = Phases(torch, stream)
        one_step(ph)
        torch.cuda.synchronize()
        for k, v in ph.durations().items():
            if not k.endswith(":start"):
                per_step.setdefault(k, []).append(v)
        log(f"[bench] step {s + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _lib.gpr_timing_enable(False)
    upd = {k: _lib.gpr_timing_read(k) for k in TIMED_KERNELS}
    per = {k: float(np.median(v)) for k, v in per_step.items()}

    # float64 check of the path against the closed-form-free reference: mixed vs float64
    res = {p: {k: outs[p][k].cpu().numpy() for k in ("alpha", "nlml", "mean", "var", "grad")} for p in precs}

    def rel(a, b):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

    summary = {}
    for p in precs:
        t_chol = per[f"{p}:cholesky"]
        train = [sum(per_step[f"{p}:{k}"][i] for k in ("assemble", "cholesky", "solve", "nlml", "grad"))
                 for i in range(args.steps)]
        pred = [per_step[f"{p}:mean"][i] + per_step[f"{p}:var"][i] for i in range(args.steps)]
        extra = {}
        if f"{p}:cholesky_device" in per:
            td = per[f"{p}:cholesky_device"]
            extra = {"cholesky_device_schedule_s": td, "cholesky_device_schedule_tflops": chol_flops(n) / td / 1e12,
                     "cholesky_device_schedule_s_spread": spread(per_step[f"{p}:cholesky_device"])}
        summary[p] = {"cholesky_s": t_chol, "cholesky_tflops": chol_flops(n) / t_chol / 1e12, **extra,
                      "cholesky_s_spread": spread(per_step[f"{p}:cholesky"]),
                      "train_step_s": float(np.median(train)), "train_step_s_spread": spread(train),
                      "predict_s": float(np.median(pred)), "predict_s_spread": spread(pred),
                      "phases_s": {k.split(":")[1]: round(v, 6) for k, v in per.items()
                                   if k.startswith(p + ":") and not k.endswith(("assemble_again", "cholesky_device"))}}
        if p != "fp64" and "fp64" in res:
            r, f = res[p], res["fp64"]
            # against the GPU's own float64 path of the same run (a proxy: that path is held to
            # the oracle by the parity tests, to 1e-10 at n = 16384 and on sampled outputs here)
            summary[p]["err_vs_fp64_gpu"] = {"mean_rel": rel(r["mean"], f["mean"]), "var_rel": rel(r["var"], f["var"]),
                                         "var_maxabs": float(np.max(np.abs(r["var"] - f["var"]))),
                                         "nlml_rel": abs(float(r["nlml"][0] - f["nlml"][0])) / abs(float(f["nlml"][0])),
                                         "alpha_rel": rel(r["alpha"], f["alpha"]),
                                         "grad_rel": rel(r["grad"], f["grad"])}
            summary[p]["speedup_cholesky_vs_fp64"] = summary["fp64"]["cholesky_s"] / t_chol
        summary[p]["nlml"] = float(res[p]["nlml"][0])

    main = "fp64" if "fp64" in summary else precs[0]
    kernels = {}
    for kind, (sym, kdt) in TIMED_KERNELS.items():
        if kind not in upd:
            continue
        cnt, ms_, fl_ = upd[kind]
        if not cnt:
            continue
        # a split-bf16 product of two float32 operands is `nprod` bf16 products: the kernel's
        # MFMA work (against the bf16 peak) is nprod times the float32-equivalent flops
        nprod = SPLIT_PRODUCTS.get(kind, 1)
        tf = nprod * fl_ / (ms_ / 1e3) / 1e12
        kernels[sym] = {"kind": kind, "role": KIND_ROLE[kind], "launches": cnt, "total_ms": round(ms_, 3),
                        "avg_launch_ms": round(ms_ / cnt, 4), "avg_launch_algo_flops": nprod * fl_ / cnt,
                        "achieved_tflops": round(tf, 4), "peak_tflops": PEAK_TFLOPS[kdt],
                        "frac": round(tf / PEAK_TFLOPS[kdt], 4), "dtype": kdt}
        if nprod > 1:
            kernels[sym]["bf16_products_per_fp32_product"] = nprod
            kernels[sym]["fp32_equivalent_tflops"] = round(tf / nprod, 4)
    for p in precs:
        k = kernels.get(TIMED_KERNELS[p][0]) if p in TIMED_KERNELS else None
        if k:
            summary[p]["update_kernel"] = {"launches": k["launches"], "avg_ms": k["avg_launch_ms"],
                                           "tflops": k["achieved_tflops"], "frac": k["frac"]}
            if "fp32_equivalent_tflops" in k:
                summary[p]["update_kernel"]["fp32_equivalent_tflops"] = k["fp32_equivalent_tflops"]
    # the dominant kernel of the float64 path: most time over the timed steps
    main_syms = [TIMED_KERNELS[k][0] for k in TIMED_KERNELS if k.split("_")[0] == main and TIMED_KERNELS[k][0] in kernels]
    dom = max(main_syms, key=lambda m: kernels[m]["total_ms"]) if main_syms else None
    dk = kernels.get(dom, {})
    line = {
        "metric": METRIC,
        "value": round(summary[main]["cholesky_tflops"], 4),   # at the median Cholesky time of the timed steps
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main == "fp64" else "f32",
        "data": "synthetic (seeded mass-spring-damper NFIR regressors)",
        "config": {"workload": f"{args.workload}: n_train={n}, n_test={m}, D={D}, tile={tile}, "
                               f"{args.kernel} kernel l=sqrt(D), nu=1, sigma^2=0.01", "precisions": precs},
        "roofline": {"bound": "mfma", "kernel": f"{dom} ({dk.get('role')})" if dom else None,
                     "achieved": dk.get("achieved_tflops"), "peak": dk.get("peak_tflops"),
                     "unit": "TFLOP/s", "frac": dk.get("frac"),
                     "traffic": recorded_traffic(dom) if dom else None, "launches": dk.get("launches"),
                     "avg_launch_ms": dk.get("avg_launch_ms"), "avg_launch_algo_flops": dk.get("avg_launch_algo_flops")},
        "kernels": kernels,
        "results": summary,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n65536_d128", choices=sorted(WORKLOADS))
    ap.add_argument("--precs", default="fp64,fp32,bf16x6,bf16x3")
    ap.add_argument("--kernel", default="se", choices=["se", "matern12", "matern32", "matern52"],
                    help="covariance function (the metric is quoted for the squared exponential)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--device-schedule", type=int, default=1,
                    help="also time the float64 factorisation under the device-side task-graph schedule (1/0)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a device copy of this many bytes (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only; the multi-GPU path is a design "
                                   "(tile-cyclic sharding) and is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()
