#!/usr/bin/env python3
"""Throughput of sketching-based Tucker-sum recompression on one MI355X.

Workload (the structured sum): d = 3, modes 512 x 512 x 512, s = 16 terms
with per-term, per-mode ranks uniform in [16, 48], cores N(0,1) scaled by
10^(-0.1 (i + j + k)), orthonormal factors; Khatri-Rao sketch, target rank
64 + oversampling 10 (m = 74).  A step is one whole recompression: Omega
generation, factor sketches, core sketches, term expansion (Y_n), FP64 thin
QR (Q_n) and core projection (H), all in the library's HIP kernels, with
inputs resident in HBM.

Forms measured (each against the FP64 oracle on the same seeded inputs):
  fp64        every stage FP64 (the plain form)
  fp32        FP32 inputs, FP32 MFMA contractions, FP64 QR
  bf16x6      FP32 inputs, split-BF16 (6 products) contractions, FP64 QR
  bf16x3      FP32 inputs, split-BF16 (3 products) sketch, bf16x6 projection
`value` is the fastest form whose end-to-end error ||X_hat - X_hat_oracle|| /
||X_hat_oracle|| is at most 1e-6.

Prints one JSON line (rank 0, one GPU).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Tucker-sum recompressions/s and % MFMA roofline vs plain FP64 at rel err <=1e-6"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2516.0}
HBM_GBS = 8000.0
FORMS = {
    # name: (input dtype, sketch precision, projection precision, output dtype)
    "fp64": ("f64", "fp64", "fp64", "f64"),
    "fp32": ("f32", "fp32", "fp32", "f32"),
    "bf16x6": ("f32", "bf16x6", "bf16x6", "f32"),
    "bf16x3": ("f32", "bf16x3", "bf16x6", "f32"),
}
PREC_CODE = {"fp64": 0, "fp32": 1, "bf16x1": 2, "bf16x3": 3, "bf16x6": 4}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--forms", default="fp64,fp32,bf16x6,bf16x3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="bound on oracle CPU time for the baseline sample")
    ap.add_argument("--profile-json", default=None, help="also write the per-kernel profile here")
    ap.add_argument("--batch-count", type=int, default=256,
                    help="sums in the batched-form leg (0 skips it)")
    return ap.parse_args()


def kernel_precision(name):
    """Arithmetic of a profiled kernel from its template arguments."""
    import re
    m = re.search(r"<(\d+)", name)
    code = int(m.group(1)) if m else 0
    return {0: "fp64", 1: "fp32", 2: "bf16x1", 3: "bf16x3", 4: "bf16x6"}.get(code, "fp64")


def kernel_peak(name):
    """(bound, peak TFLOP/s) of a contraction or QR kernel; None otherwise.
    MFMA kernels take the dense matrix peak of their arithmetic (split BF16:
    the BF16 peak over the number of products); the Cholesky and Householder
    kernels are FP64 vector arithmetic (FP64 vector peak)."""
    if "chol" in name or "householder" in name:
        return "alu", PEAK_TFLOPS["fp64"]
    if "gemm" in name or "krp" in name:
        prec = kernel_precision(name)
        if prec.startswith("bf16"):
            parts = {"bf16x1": 1, "bf16x3": 3, "bf16x6": 6}[prec]
            return "mfma", PEAK_TFLOPS["bf16"] / parts
        return "mfma", PEAK_TFLOPS[prec]
    return None


def step_roofline(report, steps, step_bytes, ms_measured):
    """Whole-step roofline: the time the step's algorithmic work needs at the
    peaks of its stages' arithmetic, or to move its algorithmic bytes,
    against the measured graph-replayed step time."""
    t_flop = 0.0
    for name, rec in report.items():
        kp = kernel_peak(name)
        if kp is not None and rec["flops"] > 0:
            t_flop += rec["flops"] / steps / (kp[1] * 1e12)
    t_bytes = step_bytes / (HBM_GBS * 1e9)
    t_roof = max(t_flop, t_bytes)
    return {"t_roof_us": t_roof * 1e6, "t_flop_us": t_flop * 1e6, "t_bytes_us": t_bytes * 1e6,
            "t_measured_us": ms_measured * 1e3, "frac": t_roof / (ms_measured * 1e-3)}


def roofline_of(report):
    """Dominant kernel (largest total time) of a profile report."""
    name, rec = max(report.items(), key=lambda kv: kv[1]["ms"])
    launches = rec["launches"]
    avg_s = rec["ms"] / launches * 1e-3
    flops = rec["flops"] / launches
    nbytes = rec["bytes"] / launches
    kp = kernel_peak(name)
    if kp is not None and kp[0] == "alu" and flops > 0:
        achieved = flops / avg_s / 1e12
        return name, {"bound": "alu", "achieved": achieved, "peak": kp[1], "unit": "TFLOP/s",
                      "frac": achieved / kp[1], "traffic": None}, avg_s
    prec = kernel_precision(name) if ("gemm" in name or "krp" in name) else None
    if prec is None or flops == 0:
        achieved = nbytes / avg_s / 1e9
        return name, {"bound": "hbm", "achieved": achieved, "peak": HBM_GBS, "unit": "GB/s",
                      "frac": achieved / HBM_GBS, "traffic": None}, avg_s
    if prec.startswith("bf16"):
        parts = {"bf16x1": 1, "bf16x3": 3, "bf16x6": 6}[prec]
        peak = PEAK_TFLOPS["bf16"] / parts   # effective rate: `parts` BF16 products per product
    else:
        peak = PEAK_TFLOPS[prec]
    ridge = peak * 1e12 / (HBM_GBS * 1e9)
    intensity = flops / max(nbytes, 1.0)
    if intensity >= ridge:
        achieved = flops / avg_s / 1e12
        return name, {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                      "frac": achieved / peak, "traffic": None}, avg_s
    achieved = nbytes / avg_s / 1e9
    return name, {"bound": "hbm", "achieved": achieved, "peak": HBM_GBS, "unit": "GB/s",
                  "frac": achieved / HBM_GBS, "traffic": None}, avg_s


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); every GPU box "
              "here has one GPU and the path has no multi-GPU part to time", file=sys.stderr)
        sys.exit(2)
    import ctypes

    import numpy as np
    import torch

    import paper_2603_13532_amd as tsk
    import synth
    from paper_2603_13532_amd import _lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    ts = synth.config_structured()
    m = ts["ell"][0]
    seed = ts["omega_seed"]
    lib = _lib.load()

    # ---- FP64 oracle on the host: reference result and CPU baseline
    from oracle import recompress as RC
    cpu = None
    t0 = time.perf_counter()
    ref = RC.recompress(ts, "krp", [m], seed)
    t_first = time.perf_counter() - t0
    runs = [t_first]
    if not args.no_cpu_baseline:
        while sum(runs) < args.cpu_seconds and len(runs) < 200:
            t0 = time.perf_counter()
            RC.recompress(ts, "krp", [m], seed)
            runs.append(time.perf_counter() - t0)
        try:
            from threadpoolctl import threadpool_info
            threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        except Exception:
            threads = os.cpu_count()
        med = float(np.median(runs))
        cpu = {"value": 1.0 / med, "unit": "recompressions/s", "cores": int(threads), "kind": "oracle",
               "sample": f"{len(runs)} full recompressions of the structured workload "
                         f"(FP64 NumPy oracle, structured path), median {med:.3f} s"}
        log(f"cpu oracle: {runs}")

    # dense reference reconstruction on the GPU (measurement only)
    def dense(h, qs):
        x = h.to(torch.float64)
        for k, q in enumerate(qs):
            q = q.to(torch.float64)
            x = torch.tensordot(x, q, dims=([0], [1]))  # contracts mode k, appends n_k last
        return x

    ref_h = torch.from_numpy(np.ascontiguousarray(ref["H"])).to(dev)
    ref_q = [torch.from_numpy(np.ascontiguousarray(q)).to(dev) for q in ref["Q"]]
    x_ref = dense(ref_h, ref_q)
    x_ref_norm = torch.linalg.vector_norm(x_ref).item()

    results = {}
    stream = torch.cuda.current_stream(dev)
    for form in [f for f in args.forms.split(",") if f]:
        in_dt, sp, pp, out_dt = FORMS[form]
        tdt = torch.float64 if in_dt == "f64" else torch.float32
        odt = torch.float64 if out_dt == "f64" else torch.float32
        cores = [tsk.fortran(torch.from_numpy(g).to(dev, tdt)) for g in ts["cores"]]
        factors = [[tsk.fortran(torch.from_numpy(u).to(dev, tdt)) for u in us] for us in ts["factors"]]
        rc = tsk.Recompressor(cores, factors, "krp", [m], seed, sketch_prec=sp, project_prec=pp,
                              out_dtype=odt)
        # eager launches (one library call per step)
        for _ in range(args.warmup):
            rc()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            rc()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_eager = ev0.elapsed_time(ev1) / args.steps
        # the same step captured once in a HIP graph and replayed
        rc.capture()
        for _ in range(args.warmup):
            rc.replay()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            rc.replay()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        qs, h = rc.replay()
        torch.cuda.synchronize()
        x = dense(h, qs)
        err = (torch.linalg.vector_norm(x - x_ref).item()) / x_ref_norm
        err_h = (torch.linalg.vector_norm(h.to(torch.float64) - ref_h) /
                 torch.linalg.vector_norm(ref_h)).item()
        del x
        ys = tsk.tucker_sum_sketch(cores, factors, "krp", [m], seed, sketch_prec=sp)
        torch.cuda.synchronize()
        err_y = max(float(np.linalg.norm(y.cpu().numpy() - yr) / np.linalg.norm(yr))
                    for y, yr in zip(ys, ref["Y"]))
        results[form] = {"ms_per_step": ms, "recompressions_per_s": 1e3 / ms,
                         "ms_per_step_eager": ms_eager,
                         "rel_err_end_to_end": err, "rel_err_H": err_h, "rel_err_Y": err_y,
                         "sketch_prec": sp, "project_prec": pp, "_rc": rc}
        log(f"{form}: {ms:.4f} ms/step graph, {ms_eager:.4f} eager, err {err:.2e} "
            f"(H {err_h:.2e}, Y {err_y:.2e})")

    # ---- batched form: 256 independent sums (uneven shapes) in one launch sequence
    batch = None
    if args.batch_count > 0:
        sums = synth.config_batch(count=args.batch_count)
        batch = {"workload": f"{args.batch_count} independent sums, d=3, n in {{64..384}}, "
                             "s in [2,10], ranks [4,40], KRP m=min(48,n/4)+8"}
        check_ids = list(range(0, len(sums), max(1, len(sums) // 8)))[:8]
        refs = {i: RC.recompress(sums[i], "krp", [sums[i]["ell"][0]], sums[i]["omega_seed"])
                for i in check_ids}
        for form in [f for f in args.forms.split(",") if f]:
            in_dt, sp, pp, out_dt = FORMS[form]
            tdt = torch.float64 if in_dt == "f64" else torch.float32
            odt = torch.float64 if out_dt == "f64" else torch.float32
            ins = []
            for one in sums:
                ins.append({"cores": [tsk.fortran(torch.from_numpy(g).to(dev, tdt)) for g in one["cores"]],
                            "factors": [[tsk.fortran(torch.from_numpy(u).to(dev, tdt)) for u in us]
                                        for us in one["factors"]],
                            "kind": "krp", "sizes": [one["ell"][0]], "seed": one["omega_seed"]})
            br = tsk.BatchRecompressor(ins, sp, pp, odt).capture()
            for _ in range(args.warmup):
                br.replay()
            torch.cuda.synchronize()
            ev0.record(stream)
            bsteps = max(3, args.steps // 5)
            for _ in range(bsteps):
                br.replay()
            ev1.record(stream)
            torch.cuda.synchronize()
            ms_b = ev0.elapsed_time(ev1) / bsteps
            qs_b, hs_b = br.replay()
            torch.cuda.synchronize()
            errs = []
            for i in check_ids:
                xr = dense(torch.from_numpy(np.ascontiguousarray(refs[i]["H"])).to(dev),
                           [torch.from_numpy(np.ascontiguousarray(q)).to(dev) for q in refs[i]["Q"]])
                xg = dense(hs_b[i], qs_b[i])
                errs.append((torch.linalg.vector_norm(xg - xr) / torch.linalg.vector_norm(xr)).item())
            batch[form] = {"ms_per_batch": ms_b, "recompressions_per_s": len(sums) * 1e3 / ms_b,
                           "max_rel_err_end_to_end_sampled": max(errs)}
            log(f"batch {form}: {ms_b:.3f} ms per {len(sums)} sums, sampled err {max(errs):.2e}")
            del br, ins

    ok = {f: r for f, r in results.items() if r["rel_err_end_to_end"] <= 1e-6}
    best = min(ok, key=lambda f: ok[f]["ms_per_step"]) if ok else "fp64"
    chosen = results[best]

    # ---- per-kernel timing of the chosen form: HIP events around every launch
    rc = chosen["_rc"]
    h = rc.h
    lib.tsk_profile_enable(h.ptr, 1)
    for _ in range(args.steps):
        rc()
    torch.cuda.synchronize()
    lib.tsk_profile_enable(h.ptr, 0)
    need = ctypes.c_size_t()
    _lib.check(lib.tsk_profile_report(h.ptr, None, 0, ctypes.byref(need)), h.ptr)
    buf = ctypes.create_string_buffer(need.value)
    _lib.check(lib.tsk_profile_report(h.ptr, buf, need.value, ctypes.byref(need)), h.ptr)
    report = json.loads(buf.value.decode())
    kname, roof, avg_s = roofline_of(report)
    roof["kernel"] = kname
    roof["avg_launch_us"] = avg_s * 1e6
    # algorithmic bytes of one step: inputs and Omega read once, Q and H written once
    in_es = 8 if FORMS[best][0] == "f64" else 4
    out_es = 8 if FORMS[best][3] == "f64" else 4
    n_in = sum(g.size for g in ts["cores"]) + sum(u.size for us in ts["factors"] for u in us)
    n_om = sum(ts["dims"][k] * m for k in range(len(ts["dims"])))
    w = min(m, min(ts["dims"]))
    n_out = sum(ts["dims"][k] * w for k in range(len(ts["dims"]))) + w ** len(ts["dims"])
    step_bytes = (n_in + n_om) * in_es + n_out * out_es
    step_roof = step_roofline(report, args.steps, step_bytes, chosen["ms_per_step"])
    if args.profile_json:
        with open(args.profile_json, "w") as f:
            json.dump({"form": best, "steps": args.steps, "report": report}, f, indent=1)

    dtype = {"fp64": "f64", "fp32": "f32", "bf16x6": "bf16x6 (f32 accumulate)",
             "bf16x3": "bf16x3/bf16x6 (f32 accumulate)"}[best]
    forms_out = {f: {k: v for k, v in r.items() if not k.startswith("_")} for f, r in results.items()}
    fp64_rate = results["fp64"]["recompressions_per_s"] if "fp64" in results else None
    line = {
        "metric": METRIC,
        "value": chosen["recompressions_per_s"],
        "unit": "recompressions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": chosen["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": "structured Tucker sum: d=3, 512^3, s=16, ranks U[16,48], "
                               "decaying Gaussian cores, orthonormal factors, KRP sketch m=74 "
                               "(target 64 + oversampling 10)",
                   "form": best, "seed": 2, "omega_seed": seed},
        "speedup_vs_plain_fp64": (chosen["recompressions_per_s"] / fp64_rate) if fp64_rate else None,
        "forms": forms_out,
        "batch_form": batch,
        "roofline": roof,
        "step_roofline": step_roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
