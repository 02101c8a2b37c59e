"""Benchmark of the visibility / chi^2 / gradient / HMC hot path on one MI355X.

Step: one leapfrog step of an HMC chain on the 61-dish hex / 49152-pixel /
lmax 100 / 64-channel / 60-time workload, run through the serving runtime:
kick + drift, sky synthesis I = Y a (separable Legendre + azimuthal stages by
default, `--synthesis dense` for the product with the stored Y), forward fringe contraction, gains +
residual + FP64 chi^2, residual collapse and gain gradient, adjoint fringe
contraction, adjoint synthesis, prior terms + kick, FP64 energy partials
(and the Metropolis test at the end of the trajectory).  The timed chain has
exactly `--steps` leapfrog steps; its initial gradient is evaluated before
timing starts.  Inputs are synthetic (seeded) and resident in HBM.  The step
rate is timed without instrumentation; a second trajectory of the same length
with HIP events around every kernel gives the per-kernel durations (the
roofline's dominant kernel) and `ms_per_step_instrumented`.

Headline value: fwd+adjoint complex MAC/s, one MAC being one term of the
fringe sum for one (unique baseline, pixel above the horizon, channel, time),
counted once for the forward and once for the adjoint contraction.

Serving (`serving` key): 64 concurrent chains on uneven hex fields
(19-127 dishes, 16-128 channels, 10-120 times, lmax 30-100), one trajectory
of 20 leapfrog steps each, through the batched server with split-precision
(bf16 hi/lo) dense synthesis and with FP32 separable synthesis (also with
dense per-channel gain mass blocks, App. B, as No-U-Turn trajectories of at
most 31 steps, and as No-U-Turn trajectories with dense gain blocks), against the
same request stream through the plain FP32 dense path one request per tick:
gradient evaluations per second and request latency p10/p50/p90/p99.

Extras (`extras` key; skipped with --no-serve unless --extras): the
delay-filtered likelihood and map-making on the timed field, with the
roofline of each one's dominant kernel, and the FP64 oracle timed beside the
GPU for both on the 16-dish workload.

Prints ONE JSON line on stdout; progress goes to stderr.
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
        "fp16_mfma_tflops": 2500.0}
EPS = 0.02   # leapfrog step in units of the diagonal-Hessian scale

# HBM bytes per launch of the fringe kernels on this workload, from two
# rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE) of
#     python3 bench.py --steps 3 --warmup 1 --no-serve --no-cpu-baseline --calibrate-copy
# each scaled by the ratio of a 256 MiB device copy's known bytes to what the
# same counter reads for it (profiles/fringe_c1_hbm_traffic.md).  The figure is
# reported only while the kernel sources and build flags hash to the value it
# was taken with.
TRAFFIC = {
    "sources": ["paper_2504_07090_amd/csrc/fringe.hip", "paper_2504_07090_amd/csrc/common.hpp",
                "paper_2504_07090_amd/build.py"],
    "sha256": "4a70a4f9bdfaf8239f323f3e473f87d5a2f626af547bdf4b32b4be21f49b12d5",
    "bytes_per_launch": {"k_fringe_adj": 195683636, "k_fringe_fwd": 235222678},
}


def sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    b = TRAFFIC["bytes_per_launch"].get(kernel)
    if b is None or TRAFFIC["sha256"] != sources_sha256(TRAFFIC["sources"]):
        return None
    return b


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# The oracle's sample of the 61-dish workload: 16 channels spread over the band
# (both ends, both 32-channel tiles of the forward kernel's map) x 2 consecutive
# times each, one (channel, time block) per single-threaded worker process.
CPU_SAMPLE_CHANNELS = [0, 4, 9, 13, 18, 22, 27, 31, 32, 36, 41, 45, 50, 54, 59, 63]
CPU_SAMPLE_TIMES = 2


def _oracle_sample(task):
    """FP64 oracle chi^2 + gradient of one (channel, time block) of the 61-dish
    workload, single-threaded; returns its MAC count, the timed seconds, and the
    model visibilities, cotangent and gradient for the GPU comparison."""
    f, t0, nt = task
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        import numpy as np
        from oracle import model
        from paper_2504_07090_amd import workload as w
        cfg = w.C1
        d = w.draw(cfg)
        fw = w.fwhm_ref_rad(cfg)
        of = model.Field(w.scaled(cfg, n_time=nt, lst0_rad=float(w.lsts(cfg)[t0])))
        m = model.forward(of, d.alm, d.gains, fw, chans=[f])
        sig = model.noise_sigma(cfg, m)
        data = m + sig * math.sqrt(2) * d.noise_unit[t0:t0 + nt, [f], :]
        t1 = time.perf_counter()
        _, ga, gg, _ = model.chi2_and_grad(of, data, sig, d.alm, d.gains, fw, chans=[f])
        t2 = time.perf_counter()
        macs = 2.0 * len(of.ubl_ij) * float(np.sum(of.up))   # forward + adjoint
        cot = -2.0 * (data - m) / sig ** 2
        return macs, t2 - t1, m[:, 0], cot[:, 0], ga[0], gg[0]


def cpu_baseline_run():
    """The oracle on a process pool over (channel, time block) samples, before the
    GPU is touched (the workers are forked).  Wall time of the pool is the
    baseline; every worker is single-threaded, so `cores` = workers."""
    import multiprocessing as mp
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    workers = max(1, min(16, ncpu, len(CPU_SAMPLE_CHANNELS)))
    tasks = [(f, (7 * k) % (60 - CPU_SAMPLE_TIMES), CPU_SAMPLE_TIMES)
             for k, f in enumerate(CPU_SAMPLE_CHANNELS)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        out = pool.map(_oracle_sample, tasks)
    wall = time.perf_counter() - t0
    macs = sum(o[0] for o in out)
    busy = sum(o[1] for o in out)
    base = {"value": macs / wall, "unit": "complex MAC/s", "cores": workers, "kind": "oracle",
            "sample": (f"FP64 NumPy oracle chi^2 + analytic gradient of {len(tasks)} (channel, "
                       f"{CPU_SAMPLE_TIMES}-time block) samples of the 61-dish workload (channels "
                       f"{CPU_SAMPLE_CHANNELS}), one single-threaded worker process per sample, "
                       f"{workers} at a time: {wall:.1f} s wall for {macs:.3e} complex MACs "
                       f"({busy:.1f} s of timed worker time; per core {macs / busy:.3e} MAC/s)")}
    return base, tasks, out


def oracle_errors(vis, torch, fld, cfg, tasks, out):
    """Per sampled channel: GPU visibilities and the GPU adjoint of the oracle's
    chi^2 cotangent against the oracle, normwise and element-wise."""
    import numpy as np
    from paper_2504_07090_amd import workload as w
    d = w.draw(cfg, with_noise=False)
    alm = torch.tensor(d.alm, dtype=torch.float32, device="cuda")
    g = torch.tensor(d.gains, dtype=torch.complex64, device="cuda")
    fw = torch.tensor([w.fwhm_ref_rad(cfg)], dtype=torch.float32, device="cuda")
    m = vis.forward(fld, alm, g, fw).cpu().numpy()
    cot = np.zeros((cfg.n_time, cfg.n_freq, fld.n_bl), dtype=np.complex64)
    for (f, t0, nt), o in zip(tasks, out):
        cot[t0:t0 + nt, f] = o[3]
    ga, gg, _ = vis.adjoint(fld, alm, g, fw, torch.tensor(cot, device="cuda"))
    ga, gg = ga.cpu().numpy(), gg.cpu().numpy()
    rows = {}
    for (f, t0, nt), o in zip(tasks, out):
        ref, got = o[2], m[t0:t0 + nt, f]
        rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
        rows[str(f)] = {
            "times": [t0, t0 + nt - 1],
            "vis_rel": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            "vis_max_over_rms": float(np.max(np.abs(got - ref)) / rms),
            "grad_alm_rel": float(np.linalg.norm(ga[f] - o[4]) / np.linalg.norm(o[4])),
            "grad_gain_rel": float(np.linalg.norm(gg[f] - o[5]) / np.linalg.norm(o[5]))}
    worst = {k: max(r[k] for r in rows.values())
             for k in ("vis_rel", "vis_max_over_rms", "grad_alm_rel", "grad_gain_rel")}
    return {"per_channel": rows, "worst": worst,
            "note": "timed field against the FP64 oracle on the cpu_baseline samples; gradients "
                    "are the adjoint of the oracle's chi^2 cotangent of each sample"}


def timed_reps(torch, fn, reps):
    """Median wall time (ms) of fn() over reps calls, each bracketed by a sync."""
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def extras_bench(vis, torch, fld, cfg, data, sigma, reps=20):
    """The delay-filtered likelihood and map-making on the timed chain's field:
    median time per call, per-kernel times (HIP events, a separate set of
    calls) and the roofline of each row's dominant kernel; the FP64 oracle and
    the GPU timed beside it on the small 16-dish workload."""
    import numpy as np
    from oracle import filter as ofl, mapmaking as omm, model
    from paper_2504_07090_amd import workload as w
    d = w.draw(cfg)
    alm = torch.tensor(d.alm, dtype=torch.float32, device="cuda")
    g = torch.tensor(d.gains, dtype=torch.complex64, device="cuda")
    fw = torch.tensor([w.fwhm_ref_rad(cfg)], dtype=torch.float32, device="cuda")
    filt = vis.Filter(w.frequencies(cfg))
    nvis = cfg.n_time * cfg.n_freq * fld.n_bl
    out = {}

    def kernel_times(fn, n=5):
        vis.profile_enable(fld, True)
        vis.profile_read(fld, reset=True)
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        kt = vis.profile_read(fld, reset=True)
        vis.profile_enable(fld, False)
        return {k: v[1] / max(1, v[0]) for k, v in kt.items()}

    # delay-filtered chi^2 + gradient: the filter GEMMs over frequency read the
    # data and model and write the weighted residual (3 x 8 B per visibility),
    # then read it and write the cotangent (2 x 8 B); 2 nf^2 flop per real
    # column and time, 10.7 flop/B: HBM-bound
    ffn = lambda: vis.chi2_filtered_and_grad(fld, filt, data, sigma, alm, g, fw)
    ffn()
    ms_f = timed_reps(torch, ffn, reps)
    kf = kernel_times(ffn)
    kr = kf.get("k_filter_resid", float("nan"))
    roof_f = {"bound": "hbm", "kernel": "k_filter_resid", "kernel_ms": kr, "unit": "GB/s",
              "achieved": 3.0 * 8.0 * nvis / (kr * 1e-3) / 1e9, "peak": PEAK["hbm_gbs"]}
    roof_f["frac"] = roof_f["achieved"] / roof_f["peak"]
    out["delay_filtered_chi2_grad"] = {"ms": ms_f, "kernel_ms": kf, "roofline": roof_f,
                                       "flop_per_launch": 2.0 * cfg.n_freq ** 2 * 2 * fld.n_bl * cfg.n_time}
    # map-making: collapse onto unique baselines, the adjoint fringe contraction
    # (same MAC count as the forward), the closed-form normalisation
    mfn = lambda: vis.make_map(fld, data, g, fw)
    mfn()
    ms_m = timed_reps(torch, mfn, reps)
    km = kernel_times(mfn)
    ka = km.get("k_fringe_adj", float("nan"))
    roof_m = {"bound": "mfma", "kernel": "k_fringe_adj", "kernel_ms": ka, "unit": "TFLOP/s",
              "achieved": 4.0 * fld.fwd_macs / (ka * 1e-3) / 1e12, "peak": PEAK["fp32_mfma_tflops"]}
    roof_m["frac"] = roof_m["achieved"] / roof_m["peak"]
    out["map_making"] = {"ms": ms_m, "kernel_ms": km, "roofline": roof_m}
    # the oracle beside the GPU on the 16-dish workload (8 channels, 4 times)
    c0 = w.C0
    b0 = vis.basis_for(c0)
    f0 = vis.Field.from_config(b0, c0)
    of = model.Field(c0)
    d0 = w.draw(c0)
    _, s0, y0 = model.make_data(of, d0)
    fr0 = w.frequencies(c0)
    t0 = time.perf_counter()
    ofl.chi2_filtered_and_grad(of, y0, s0, ofl.delay_filter(fr0), d0.alm, d0.gains, w.fwhm_ref_rad(c0))
    t_of = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    omm.dirty_map(of, y0, d0.gains, w.fwhm_ref_rad(c0))
    t_om = (time.perf_counter() - t0) * 1e3
    a0 = torch.tensor(d0.alm, dtype=torch.float32, device="cuda")
    g0 = torch.tensor(d0.gains, dtype=torch.complex64, device="cuda")
    fw0 = torch.tensor([w.fwhm_ref_rad(c0)], dtype=torch.float32, device="cuda")
    y0d = torch.tensor(np.ascontiguousarray(y0), dtype=torch.complex64, device="cuda")
    filt0 = vis.Filter(fr0)
    g_of = timed_reps(torch, lambda: vis.chi2_filtered_and_grad(f0, filt0, y0d, s0, a0, g0, fw0), reps)
    g_om = timed_reps(torch, lambda: vis.make_map(f0, y0d, g0, fw0), reps)
    out["oracle_beside_gpu_16dish"] = {
        "workload": c0.name, "unit": "ms per call",
        "delay_filtered_chi2_grad": {"oracle_ms": t_of, "gpu_ms": g_of},
        "map_making": {"oracle_ms": t_om, "gpu_ms": g_om}}
    return out


def make_chain(vis, serve, torch, basis, cfg, prec, synthesis=0):
    """Field, synthetic data, inverse mass and prior for one chain of config cfg."""
    from paper_2504_07090_amd import workload as w
    fld = vis.Field.from_config(basis, cfg, prec, synthesis)
    d = w.draw(cfg)
    alm = torch.tensor(d.alm, dtype=torch.float32, device="cuda")
    g = torch.tensor(d.gains, dtype=torch.complex64, device="cuda")
    fw = torch.tensor([w.fwhm_ref_rad(cfg)], dtype=torch.float32, device="cuda")
    m = vis.forward(fld, alm, g, fw)
    rms = float(torch.sqrt(torch.mean(m.abs().double() ** 2)))
    sigma = cfg.noise_frac * rms / math.sqrt(2.0)
    data = (m + sigma * math.sqrt(2.0) * torch.tensor(d.noise_unit, dtype=torch.complex64,
                                                      device="cuda")).contiguous()
    del m
    lay = serve.Layout(fld)
    cvar = torch.tensor(d.alm_var, dtype=torch.float32, device="cuda")
    _, minv = serve.mass_diag(fld, alm, g, fw, sigma, cvar, cfg.gain_scatter, n_probes=16)
    # start slightly off the truth: 1% of the prior width
    gen = torch.Generator(device="cuda")
    gen.manual_seed(cfg.seed)
    q0 = lay.pack(alm, g, fw)
    q0[:lay.nalm] += 0.01 * torch.sqrt(cvar.reshape(-1)) * torch.randn(lay.nalm, generator=gen,
                                                                       device="cuda")
    return fld, data, sigma, q0.contiguous(), minv, cvar, lay


def wait_requests(srv, n, timeout_s=300):
    t_end = time.monotonic() + timeout_s
    while srv.stats()["requests"] < n:
        if time.monotonic() > t_end:
            raise TimeoutError("server did not finish the initial evaluations")
        time.sleep(0.002)


def serving_inputs(vis, serve, torch, basis, n_chains):
    """Per-chain configs, data, start points and mass matrices (made once, FP32 fields)."""
    from paper_2504_07090_amd import workload as w
    out = []
    for c in range(n_chains):
        cfg = w.serving_chain_config(c)
        fld, data, sigma, q0, minv, cvar, lay = make_chain(vis, serve, torch, basis, cfg,
                                                           vis.VIS_FP32)
        out.append((cfg, fld, data, sigma, q0, minv, cvar))
    return out


def serving_bench(vis, serve, torch, basis, inputs, prec, max_batch, n_leapfrog=20, synthesis=0,
                  dense_gains=False, nuts_depth=0, batched=None):
    """One trajectory of n_leapfrog steps per chain; all chains submitted at once.
    dense_gains: every chain gets dense per-channel gain mass blocks (the
    Gauss-Newton gain Hessian plus the prior, built before timing).
    nuts_depth > 0: one No-U-Turn trajectory per chain instead (at most
    2^nuts_depth - 1 steps, ended by the device)."""
    n_chains = len(inputs)
    flds = [f if (prec == vis.VIS_FP32 and synthesis == 0)
            else vis.Field.from_config(basis, cfg, prec, synthesis)
            for (cfg, f, *_rest) in inputs]
    chols = [None] * n_chains
    if dense_gains:
        for c, ((cfg, _, data, sigma, q0, minv, cvar), fld) in enumerate(zip(inputs, flds)):
            alm, g, fw = serve.Layout(fld).unpack(q0)
            chols[c] = serve.gain_mass_blocks(fld, alm.contiguous(), g.contiguous(),
                                              fw.contiguous(), sigma, cfg.gain_scatter)
    fp = sum(serve.Server.footprint(f, dense_gains, nuts_depth > 0) for f in flds)
    if batched is None:
        batched = 1 if max_batch > 1 else 0
    srv = serve.Server(fp + (64 << 20), max_chains=n_chains, max_batch=max_batch, batched=batched)
    ids = []
    for c, ((cfg, _, data, sigma, q0, minv, cvar), fld) in enumerate(zip(inputs, flds)):
        ids.append(srv.admit(fld, data, sigma, q0, minv, cvar, cfg.gain_scatter, EPS, n_leapfrog,
                             seed=7, stream_id=c, adapt_step=True, gain_chol=chols[c],
                             nuts_max_depth=nuts_depth))
    wait_requests(srv, n_chains)
    srv.stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in ids:
        srv.submit(i, 1)
    res = srv.wait(n_chains, timeout_s=600)
    t1 = time.perf_counter()
    if any(r["status"] != 0 for r in res):
        raise RuntimeError("a serving chain failed: " + str([r for r in res if r["status"]][:2]))
    st = srv.stats()
    srv.close()
    by_chain = {i: c for c, i in enumerate(ids)}
    # leapfrog steps that belong to trajectories (a NUTS chain also runs up to
    # two no-op steps between the device's end of a trajectory and the host's
    # next start; those count in "requests" but not here)
    steps = [r["n_grad"] for r in res]
    macs = sum(2.0 * flds[by_chain[r["chain"]]].fwd_macs * r["n_grad"] for r in res)
    acc = sum(r["accepted"] for r in res) / len(res)
    out = {"grad_evals_per_s": st["requests"] / (t1 - t0), "p10_ms": st["p10_ms"],
           "p50_ms": st["p50_ms"], "p90_ms": st["p90_ms"], "p99_ms": st["p99_ms"],
           "requests": st["requests"], "wall_s": t1 - t0,
           "complex_macs_per_s": macs / (t1 - t0), "acceptance": acc, "max_batch": max_batch,
           "evaluation_launches": {0: "one chain after another", 1: "batched grids",
                                   2: "per chain on several streams"}[batched]}
    if nuts_depth:
        out.update({"trajectory_grad_evals_per_s": sum(steps) / (t1 - t0),
                    "mean_steps": sum(steps) / len(steps), "max_depth": nuts_depth,
                    "depths": sorted(r["tree_depth"] for r in res)[::max(1, len(res) // 8)]})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--serve-precision", default="bf16x3", choices=["bf16x3", "fp16x3"])
    ap.add_argument("--synthesis", default="separable", choices=["separable", "dense"],
                    help="sky synthesis of the timed chain (separable: FP32 only)")
    ap.add_argument("--serve-chains", type=int, default=64)
    ap.add_argument("--inflight-ticks", type=int, default=1, choices=[1, 2],
                    help="serving ticks in flight for the timed chain (2: the next tick is "
                         "built and queued while the current one runs)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-modes", default="split,split_separable,separable,multistream,"
                    "dense_gains,nuts,nuts_dense_gains,per_chain",
                    help="serving runs to measure (comma list; the speed-ups need split, "
                         "separable and per_chain)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the delay-filtered likelihood and map-making measurements "
                         "(also skipped with --no-serve, as in the profiling runs)")
    ap.add_argument("--extras", action="store_true",
                    help="run those measurements even with --no-serve")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with a 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    cpu = samples = None
    if not args.no_cpu_baseline:
        # before the GPU is initialised: the pool forks
        log("cpu baseline (oracle on a process pool over channel / time samples)")
        cpu, sample_tasks, sample_out = cpu_baseline_run()
        samples = (sample_tasks, sample_out)

    import torch
    from paper_2504_07090_amd import serve, vis, workload as w

    torch.cuda.set_device(0)
    cfg = w.C1
    precs = {"fp32": vis.VIS_FP32, "bf16x3": vis.VIS_BF16X3, "fp16x3": vis.VIS_FP16X3}
    prec = precs[args.precision]
    sprec = precs[args.serve_precision]
    synth = vis.VIS_SYNTH_SEPARABLE if args.synthesis == "separable" else vis.VIS_SYNTH_DENSE
    log("basis + fields", cfg.name, args.synthesis, "synthesis")
    storage = (vis.STORAGE_SEPARABLE if synth == vis.VIS_SYNTH_SEPARABLE else vis.STORAGE_FOR[prec]) | \
        (0 if args.no_serve else 1 | vis.STORAGE_FOR[sprec] | vis.STORAGE_SEPARABLE)
    basis = vis.basis_for(cfg, storage=storage)
    warm = make_chain(vis, serve, torch, basis, cfg, prec, synth)
    timed = make_chain(vis, serve, torch, basis, cfg, prec, synth)
    fld = timed[0]
    # one chain per tick: its kernels launch one by one (batched=0), so the
    # per-field kernel timers can bracket each of them
    srv = serve.Server(serve.Server.footprint(fld) * 2 + (64 << 20), max_chains=2, max_batch=2,
                       batched=0, inflight_ticks=args.inflight_ticks)
    fldw, dataw, sigw, q0w, minvw, cvarw, _ = warm
    cw = srv.admit(fldw, dataw, sigw, q0w, minvw, cvarw, cfg.gain_scatter, EPS,
                   max(1, args.warmup), seed=1, stream_id=0)
    srv.submit(cw, 1)
    srv.wait(1, timeout_s=300)
    fld, data, sigma, q0, minv, cvar, lay = timed
    ct = srv.admit(fld, data, sigma, q0, minv, cvar, cfg.gain_scatter, EPS, args.steps,
                   seed=2, stream_id=1)
    wait_requests(srv, 1 + max(1, args.warmup) + 1)   # warm-up chain + the timed chain's initial gradient
    srv.stats(reset=True)
    log("timed trajectory of", args.steps, "leapfrog steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    srv.submit(ct, 1)
    res = srv.wait(1, timeout_s=600)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = srv.stats()
    # Per-kernel durations come from a second trajectory of the same length
    # with a HIP event pair around every kernel of the evaluation; the events
    # idle the GPU for a few microseconds at each kernel boundary, so the step
    # rate above is taken without them.
    log("instrumented trajectory (per-kernel HIP events)")
    vis.profile_enable(fld, True)
    vis.profile_read(fld, reset=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    srv.submit(ct, 1)
    res2 = srv.wait(1, timeout_s=600)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ktimes = vis.profile_read(fld, reset=True)
    vis.profile_enable(fld, False)
    srv.close()
    for r in (res[0], res2[0]):
        if r["status"] != 0:
            raise RuntimeError(f"timed chain failed: {r}")
    ms = (t1 - t0) * 1e3 / args.steps
    ms_instr = (t3 - t2) * 1e3 / args.steps
    macs = 2.0 * fld.fwd_macs
    value = macs / (ms * 1e-3)
    log("ms/step", ms, "result", res[0])

    per = {k: v[1] / max(1, v[0]) for k, v in ktimes.items()}
    dom = max(ktimes, key=lambda k: ktimes[k][1])
    dom_ms = per[dom]
    nv = fld.info.n_pix_visible
    if dom.startswith("k_fringe"):
        work = 4.0 * fld.fwd_macs            # 2 FMA per complex x real MAC
        # split-precision fields run both fringe GEMMs on FP16 MFMA
        roof = {"bound": "mfma", "peak": PEAK["fp32_mfma_tflops"] if prec == vis.VIS_FP32
                else PEAK["fp16_mfma_tflops"]}
    else:
        work = 2.0 * cfg.n_freq * nv * fld.n_modes
        roof = {"bound": "mfma", "peak": PEAK["fp32_mfma_tflops"] if prec == vis.VIS_FP32
                else PEAK["bf16_mfma_tflops"]}
    roof.update({"achieved": work / (dom_ms * 1e-3) / 1e12, "unit": "TFLOP/s"})
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom) if prec == vis.VIS_FP32 else None
    roof["kernel"] = dom
    roof["kernel_ms"] = dom_ms

    extras = None
    if args.extras or (not args.no_serve and not args.no_extras):
        log("extras: delay-filtered likelihood and map-making on the timed field")
        extras = extras_bench(vis, torch, fld, cfg, data, sigma)

    serving = None
    if not args.no_serve:
        log("serving: building", args.serve_chains, "uneven chains")
        ins = serving_inputs(vis, serve, torch, basis, args.serve_chains)
        modes = set(args.serve_modes.split(","))
        runs = {}

        def sb(name, label, **kw):
            if name in modes:
                log("serving:", label)
                runs[name] = serving_bench(vis, serve, torch, basis, ins, **kw)

        sb("split", f"batched, {args.serve_precision}, dense synthesis", prec=sprec,
           max_batch=args.serve_chains)
        sb("split_separable", "batched, FP32 separable synthesis, fp16x3 fringe",
           prec=vis.VIS_FP16X3, max_batch=args.serve_chains, synthesis=vis.VIS_SYNTH_SEPARABLE)
        sb("separable", "batched, FP32 separable synthesis", prec=vis.VIS_FP32,
           max_batch=args.serve_chains, synthesis=vis.VIS_SYNTH_SEPARABLE)
        sb("multistream", "FP32 separable synthesis, each chain's kernels on their own (4 streams)",
           prec=vis.VIS_FP32, max_batch=args.serve_chains, synthesis=vis.VIS_SYNTH_SEPARABLE,
           batched=2)
        sb("dense_gains", "batched, FP32 separable synthesis, dense gain mass blocks",
           prec=vis.VIS_FP32, max_batch=args.serve_chains, synthesis=vis.VIS_SYNTH_SEPARABLE,
           dense_gains=True)
        sb("nuts", "batched, FP32 separable synthesis, NUTS (at most 5 doublings)",
           prec=vis.VIS_FP32, max_batch=args.serve_chains, synthesis=vis.VIS_SYNTH_SEPARABLE,
           nuts_depth=5)
        sb("nuts_dense_gains", "batched, FP32 separable synthesis, NUTS with dense gain mass blocks",
           prec=vis.VIS_FP32, max_batch=args.serve_chains, synthesis=vis.VIS_SYNTH_SEPARABLE,
           dense_gains=True, nuts_depth=5)
        sb("per_chain", "per-chain FP32 baseline (dense synthesis), one request per tick",
           prec=vis.VIS_FP32, max_batch=1)
        del ins
        names = {"split": "batched_" + args.serve_precision,
                 "split_separable": "batched_fp16x3_fringe_separable",
                 "separable": "batched_fp32_separable",
                 "multistream": "multistream_fp32_separable",
                 "dense_gains": "batched_fp32_separable_dense_gain_mass",
                 "nuts": "batched_fp32_separable_nuts",
                 "nuts_dense_gains": "batched_fp32_separable_nuts_dense_gain_mass",
                 "per_chain": "per_chain_fp32"}
        serving = {"chains": args.serve_chains, "leapfrog_steps": 20}
        serving.update({names[k]: v for k, v in runs.items()})
        if "per_chain" in runs:
            base = runs["per_chain"]["grad_evals_per_s"]
            if "split" in runs:
                serving["speedup"] = runs["split"]["grad_evals_per_s"] / base
            if "separable" in runs:
                serving["speedup_separable"] = runs["separable"]["grad_evals_per_s"] / base
            if "split_separable" in runs:
                serving["speedup_split_separable"] = runs["split_separable"]["grad_evals_per_s"] / base

    errors = None
    if samples is not None:
        log("errors against the oracle on its samples")
        errors = oracle_errors(vis, torch, fld, cfg, *samples)

    line = {
        "metric": "fwd+adjoint complex MAC/s; batched-HMC grad evals/s + p50/p99 latency",
        "value": value, "unit": "complex MAC/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec == vis.VIS_FP32 else args.precision,
        "data": "synthetic",
        "config": {"workload": cfg.name, "synthesis": args.synthesis,
                   "n_ant": fld.n_ant, "n_bl": fld.n_bl, "n_ubl": fld.n_ubl,
                   "n_pix": fld.info.n_pix, "n_pix_visible": nv, "lmax": cfg.lmax,
                   "n_freq": cfg.n_freq, "n_time": cfg.n_time, "fwd_macs": fld.fwd_macs,
                   "leapfrog_steps": args.steps, "inflight_ticks": args.inflight_ticks},
        "grad_evals_per_s": 1e3 / ms,
        "ms_per_step_instrumented": ms_instr,
        "p10_ms": st["p10_ms"], "p50_ms": st["p50_ms"], "p90_ms": st["p90_ms"],
        "p99_ms": st["p99_ms"],
        "kernel_ms": per,
        "roofline": roof,
        "serving": serving,
        "extras": extras,
        "error_vs_oracle": errors,
        "cpu_baseline": cpu,
    }
    if args.calibrate_copy:
        # reference for the HBM byte counters: 256 MiB read + 256 MiB written
        x = torch.empty(64 << 20, dtype=torch.float32, device="cuda").uniform_()
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    print(json.dumps(line))


if __name__ == "__main__":
    main()
