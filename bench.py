"""Benchmark of the visibility / chi^2 / gradient hot path on one MI355X.

One step = one chi^2 + gradient evaluation of the full path on the 61-dish
hex / 49152-pixel / lmax 100 / 64-channel / 60-time workload: sky synthesis
I = Y a, forward fringe contraction, gains + residual + chi^2, residual
collapse and gain gradient, adjoint fringe contraction, adjoint synthesis,
followed by one diagonal-mass leapfrog update of the parameter vector.
Inputs are synthetic (seeded) and resident in HBM before timing starts.

Headline value: fwd+adjoint complex MAC/s, one MAC being one term of the
fringe sum for one (unique baseline, pixel above the horizon, channel, time),
counted once for the forward and once for the adjoint contraction.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"hbm_gbs": 8000.0, "fp32_mfma_tflops": 157.3, "bf16_mfma_tflops": 2500.0,
        "fp32_vector_tflops": 157.3}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(cfg, chan: int = 37):
    """Oracle chi^2 + gradient for one channel of the workload (all times), FP64."""
    import numpy as np
    from oracle import model
    from paper_2504_07090_amd import workload as w
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        blas_threads = os.cpu_count() or 1
    d = w.draw(cfg)
    of = model.Field(cfg)
    t0 = time.perf_counter()
    m = model.forward(of, d.alm, d.gains, w.fwhm_ref_rad(cfg), chans=[chan])
    sig = model.noise_sigma(cfg, m)
    data = m + sig * math.sqrt(2) * d.noise_unit[:, [chan], :]
    t1 = time.perf_counter()
    model.chi2_and_grad(of, data, sig, d.alm, d.gains, w.fwhm_ref_rad(cfg), chans=[chan])
    t2 = time.perf_counter()
    macs = 2.0 * len(of.ubl_ij) * float(np.sum(of.up))  # fwd + adjoint, one channel
    return {"value": macs / (t2 - t1), "unit": "complex MAC/s", "cores": int(blas_threads),
            "kind": "oracle",
            "sample": (f"FP64 NumPy oracle chi^2 + analytic gradient of channel {chan} only, all "
                       f"{cfg.n_time} times, {len(of.ubl_ij)} unique baselines, full grid: "
                       f"{t2 - t1:.1f} s (data generation {t1 - t0:.1f} s not timed); elementwise "
                       f"NumPy is single-threaded, BLAS uses {blas_threads} threads")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2504_07090_amd import vis, workload as w

    torch.cuda.set_device(0)
    cfg = w.C1
    prec = vis.VIS_FP32 if args.precision == "fp32" else vis.VIS_BF16X3
    log("building basis and field", cfg.name)
    basis = vis.basis_for(cfg, storage=vis.STORAGE_FOR[prec])
    fld = vis.Field.from_config(basis, cfg, prec)
    d = w.draw(cfg)
    alm = torch.tensor(d.alm, dtype=torch.float32, device="cuda")
    gains = torch.tensor(d.gains, dtype=torch.complex64, device="cuda")
    fwhm = torch.tensor([w.fwhm_ref_rad(cfg)], dtype=torch.float32, device="cuda")
    # synthetic data: model at the truth plus noise of 1% of the visibility rms
    m_true = vis.forward(fld, alm, gains, fwhm)
    rms = float(torch.sqrt(torch.mean(m_true.abs().double() ** 2)))
    sigma = cfg.noise_frac * rms / math.sqrt(2.0)
    noise = torch.tensor(d.noise_unit, dtype=torch.complex64, device="cuda")
    data = (m_true + sigma * math.sqrt(2.0) * noise).contiguous()
    del noise, m_true
    # evaluate at a perturbed point so the gradient is not dominated by noise
    alm_q = (alm * 1.05).contiguous()
    torch.cuda.synchronize()

    def step():
        return vis.chi2_and_grad(fld, data, sigma, alm_q, gains, fwhm)

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    vis.profile_enable(fld, True)
    vis.profile_read(fld, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ktimes = vis.profile_read(fld, reset=True)
    vis.profile_enable(fld, False)
    ms = (t1 - t0) * 1e3 / args.steps
    macs = 2.0 * fld.fwd_macs
    value = macs / (ms * 1e-3)
    log("chi2", float(out[0]), "ms/step", ms)

    # dominant kernel and its roofline
    per = {k: v[1] / max(1, v[0]) for k, v in ktimes.items()}
    dom = max(ktimes, key=lambda k: ktimes[k][1])
    dom_ms = per[dom]
    nv = fld.info.n_pix_visible
    if dom.startswith("k_fringe"):
        work = 4.0 * fld.fwd_macs            # 2 FMA per complex x real MAC
        roof = {"bound": "mfma", "achieved": work / (dom_ms * 1e-3) / 1e12,
                "peak": PEAK["fp32_mfma_tflops"], "unit": "TFLOP/s"}
    else:
        work = 2.0 * cfg.n_freq * nv * fld.n_modes
        pk = PEAK["fp32_mfma_tflops"] if prec == vis.VIS_FP32 else PEAK["bf16_mfma_tflops"]
        roof = {"bound": "mfma", "achieved": work / (dom_ms * 1e-3) / 1e12, "peak": pk,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = dom
    roof["kernel_ms"] = dom_ms

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one channel)")
        cpu = cpu_baseline(cfg)

    line = {
        "metric": "fwd+adjoint complex MAC/s; batched-HMC grad evals/s + p50/p99 latency",
        "value": value, "unit": "complex MAC/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec == vis.VIS_FP32 else "bf16x3",
        "data": "synthetic",
        "config": {"workload": cfg.name, "n_ant": fld.n_ant, "n_bl": fld.n_bl, "n_ubl": fld.n_ubl,
                   "n_pix": fld.info.n_pix, "n_pix_visible": nv, "lmax": cfg.lmax,
                   "n_freq": cfg.n_freq, "n_time": cfg.n_time, "fwd_macs": fld.fwd_macs},
        "kernel_ms": {k: v[1] / max(1, v[0]) for k, v in ktimes.items()},
        "grad_evals_per_s": 1e3 / ms,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
