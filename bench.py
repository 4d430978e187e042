#!/usr/bin/env python3
"""Benchmark of the FCH pseudo-spectral BDF2 hot path on one MI355X.

Headline: fixed-step BDF2-IMEX steps/s on the 1024^2 FP64 workload (one
circular bilayer on [0, 16 pi]^2, eps = 0.1, k = 1e-3), inputs resident in
HBM.  A step is one chemical-potential evaluation (4 real 2D transforms with
the pointwise well fused in) plus the IMEX diagonal solve, run as the fused
launch chain (row pass, column pass) of the library.

The same JSON line carries:
  roofline     -- the dominant kernel's algorithmic bytes per launch over its
                  average duration in the timed steps (each launch records its
                  start on the device clock; a kernel's time is the interval to
                  the next launch's start in the back-to-back chain), against
                  8 TB/s; traffic from the committed rocprofv3 FETCH_SIZE /
                  WRITE_SIZE summary when it was taken on the current kernel
                  source and on the variant the run timed;
  roofline_streaming -- the same for the 2048^2 adaptive PSD run (working set
                  beyond the 256 MB Infinity Cache), traffic from its own
                  counter summary (--streaming-only runs that leg alone);
  cpu_baseline -- the CPU oracle on a bounded sample of the same workload;
  extra        -- SAV, ETDRK2 and adaptive steps/s, PSD iterations/s and FFT
                  calls per PSD step, 2D FFT GB/s on a 32-field batch, the
                  critical-d sweep, the ensembles and the learned warm start
                  (trained in the run at reduced scale, and from stored
                  full-scale parameters on full-length held-out runs).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def spec_bytes(N):
    return 16 * N * (N // 2 + 1)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fch_device.hpp", "fch_kernels_impl.hpp", "fch_coef.hpp"):
        with open(os.path.join(ROOT, "paper_2006_04784_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def row_kernel_name(N, cfg):
    """Name of the row pass (chemical-potential mode) of launch config cfg =
    (row R, row E, row twl, col E, col twl), as rocprofv3 reports it."""
    return "fch::k_row<%d, %d, %d, 0, %d>" % (N, cfg[0], cfg[1], cfg[2])


def read_traffic(kernel_class, summary="pmc_traffic_m1_imex.txt", kernel=None):
    """HBM bytes per launch from a committed counter summary, if it was
    taken on the current kernel source and, when `kernel` is given, on that
    kernel (else None)."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        m = re.match(r"\s*([a-z_0-9]+)\s*:\s*(.+?)\s*$", line)
        if m:
            kv[m.group(1)] = m.group(2)
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    if kernel is not None and kv.get("%s_kernel" % kernel_class) != kernel:
        return None
    key = "%s_bytes_per_launch" % kernel_class
    return float(kv[key]) if key in kv else None


def hbm_roofline(kernels, label, extra=None, where="the timed region"):
    """Roofline object of the dominant kernel (largest total time) among
    kernels = {name: (algorithmic bytes per launch, avg seconds, launches)}."""
    dom = max(kernels, key=lambda kk: kernels[kk][1] * kernels[kk][2])
    nbytes, avg, count = kernels[dom]
    achieved = nbytes / avg / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
           "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
           "kernel": dom, "workload": label, "bytes_per_launch": nbytes,
           "avg_us": round(avg * 1e6, 3),
           "timing": "device clock in %s: start of each launch to the next launch's start "
                     "in the back-to-back chain, %d launches" % (where, count),
           "other_kernels": {kk: {"avg_us": round(v[1] * 1e6, 3), "bytes_per_launch": v[0],
                                  "GBps": round(v[0] / v[1] / 1e9, 1), "launches": v[2]}
                             for kk, v in kernels.items()}}
    out.update(extra or {})
    return out


def prof_kernels(prof, row_bytes, col_bytes, col_name):
    """(bytes, avg seconds, launches) of the row pass and the fused column pass
    from a plan's mode-2 kernel timing (fch_plan_profile_read)."""
    rn, rms = prof["row_mu"]
    cn, cms = prof["col_fused"]
    return {"row_mu": (row_bytes, rms * 1e-3 / max(rn, 1), rn),
            col_name: (col_bytes, cms * 1e-3 / max(cn, 1), cn)}


def c3_leg(dev):
    """c3: 2048^2 adaptive BDF2-PSD, its extra entry and the streaming roofline."""
    import torch

    from paper_2006_04784_amd import fch, inputs
    # c3: 2048^2 adaptive BDF2-PSD (i_tol 1e-10, LTE target 1e-6, k_max 0.05), the
    # first 100 accepted steps after the startup step
    log("c3: 2048^2 adaptive BDF2-PSD, 100 accepted steps")
    kw3, u3 = inputs.workload("c3")
    plan3 = fch.Plan(**kw3, device=dev)
    a3 = plan3.forward(torch.from_numpy(u3).to(dev))
    b3 = torch.empty_like(a3)
    u3d = a3.clone()
    plan3.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info3 = plan3.run(a3, b3, scheme="psd", adaptive=True, startup=True, t_end=100.0,
                      nsteps=101, k_first=1e-6,
                      adapt=fch.AdaptOpts(sigma_tol=1e-6, k_max=0.05), psd_tol=1e-10)
    torch.cuda.synchronize()
    el3 = time.perf_counter() - t0
    S3 = spec_bytes(kw3["N"])
    acc3 = info3["accepted"]
    launches3 = plan3.stats()["launches"]
    # the same run with kernel timing on (each row and column pass records
    # its start on the device clock; attempts then run from the host loop,
    # one host wait per chunk of PSD iterations and per error estimate)
    a3.copy_(u3d)
    plan3.profile(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info3h = plan3.run(a3, b3, scheme="psd", adaptive=True, startup=True, t_end=100.0,
                       nsteps=101, k_first=1e-6,
                       adapt=fch.AdaptOpts(sigma_tol=1e-6, k_max=0.05), psd_tol=1e-10)
    torch.cuda.synchronize()
    el3h = time.perf_counter() - t0
    prof3 = plan3.profile_read()
    plan3.profile(False)
    c3 = {
        "accepted_steps": acc3, "rejected": info3["rejected"], "t": round(info3["t"], 6),
        "psd_iters_per_step": round(info3["psd_iters"] / acc3, 2),
        "psd_fft_calls_per_step": round(4.0 * info3["psd_iters"] / acc3, 2),
        "total_fft_calls_per_step": round(info3["fft_calls"] / acc3, 2),
        "ms_per_step": round(1e3 * el3 / acc3, 3),
        "launches_per_step": round(launches3 / acc3, 2),
        "control": "device (queued rounds, one host wait per 8 rounds)",
        "ms_per_step_host_loop_timed": round(1e3 * el3h / info3h["accepted"], 3),
        "psd_iteration_GBps": round(11 * S3 * info3["psd_iters"] / el3 / 1e9, 1),
        "bytes_per_psd_iteration": 11 * S3}
    # streaming roofline: the kernels of the timed rerun (working set: u^n, u^{n-1},
    # the iterate, b u^n + c u^{n-1}, the pair buffer and three F caches,
    # 9S = 302 MB, beyond the 256 MB Infinity Cache); row passes of the PSD
    # iterations and of the error estimate, PSD column passes
    kern3 = prof_kernels(prof3, 4 * S3, 7 * S3, "col_psd_fused")
    roofline_streaming = hbm_roofline(
        kern3, "c3 2048^2 adaptive BDF2-PSD, first 100 accepted steps (40 loops + random "
               "field, working set 9S = %.0f MB)" % (9 * S3 / 1e6),
        {"iteration_bytes": 11 * S3,
         "iteration_frac": round(11 * S3 / (kern3["row_mu"][1] + kern3["col_psd_fused"][1])
                                 / 1e9 / PEAK_HBM_GBS, 4)},
        where="the run's rerun with kernel timing on")
    roofline_streaming["traffic"] = read_traffic(
        roofline_streaming["kernel"], "pmc_traffic_c3_psd.txt",
        row_kernel_name(kw3["N"], plan3.get_config())
        if roofline_streaming["kernel"] == "row_mu" else None)
    del plan3, a3, b3
    return c3, roofline_streaming


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip SAV/PSD/adaptive/FFT extras")
    ap.add_argument("--streaming-only", action="store_true",
                    help="of the extras run only the 2048^2 PSD leg (for counter runs)")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="of the extras, run only the two batched ensembles (for profiling)")
    ap.add_argument("--config", type=str, default="",
                    help="row_R,row_E,row_twl,col_E,col_twl launch config instead of autotuning")
    ap.add_argument("--graph", type=int, default=0,
                    help="steps per HIP-graph replay of the fused IMEX chain (0: launch each kernel)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB copy (counter calibration)")
    args = ap.parse_args()
    if args.streaming_only:
        args.no_extra = True  # the 2048^2 PSD leg runs alone
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2006_04784_amd import fch, inputs

    dev = torch.device("cuda:0")
    kw, u0 = inputs.workload("m1")
    N = kw["N"]
    k = 1e-3
    plan = fch.Plan(**kw, device=dev)
    S = spec_bytes(N)

    log("m1 1024^2: forward transform and startup step")
    uh0 = plan.forward(torch.from_numpy(u0).to(dev))
    a, b = uh0.clone(), torch.empty_like(uh0)
    plan.run(a, b, scheme="imex", nsteps=1, k=k, startup=True)
    if args.config:
        plan.set_config(tuple(int(x) for x in args.config.split(",")))
        log("launch config %s (given)" % (plan.get_config(),))
    else:
        log("autotune launch variants")
        tuned_cfg, tuned_us = plan.autotune(a, b, k=k, reps=20)
        log("chosen %s (row %.2f us, column %.2f us)" % (tuned_cfg, tuned_us[0], tuned_us[1]))
    plan.set_graph(args.graph)
    log("warmup %d steps (graph replay of %d steps)" % (args.warmup, args.graph))
    plan.run(a, b, scheme="imex", nsteps=args.warmup, k=k, k_prev=k, startup=False)
    torch.cuda.synchronize()

    # the timed steps also carry the kernel timing (each launch's start on the
    # device clock; nothing is added to the stream)
    log("timed %d steps" % args.steps)
    plan.profile(2)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    plan.run(a, b, scheme="imex", nsteps=args.steps, k=k, k_prev=k, startup=False)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile_read()
    plan.profile(False)
    dt = t1 - t0
    steps_per_s = args.steps / dt
    ms_per_step = 1e3 * dt / args.steps
    if not torch.isfinite(a).all():
        raise RuntimeError("non-finite state after the timed run")

    # ---- roofline: the dominant kernel of the timed steps -------------------
    kern = prof_kernels(prof, 4 * S, 7 * S, "col_imex_fused")
    roofline = hbm_roofline(kern, "m1 1024^2 fixed-step BDF2-IMEX", {
        "step_bytes": 11 * S,
        "step_us_events": round(ev0.elapsed_time(ev1) * 1e3 / args.steps, 3),
        "step_GBps": round(11 * S * steps_per_s / 1e9, 1),
        "step_frac": round(11 * S * steps_per_s / 1e9 / PEAK_HBM_GBS, 4)})
    roofline["traffic"] = read_traffic(
        roofline["kernel"], kernel=row_kernel_name(N, plan.get_config())
        if roofline["kernel"] == "row_mu" else None)

    extra = {}
    roofline_streaming = None
    if args.streaming_only:
        c3, roofline_streaming = c3_leg(dev)
        extra["c3_psd_adaptive_2048"] = c3
    elif not args.no_extra and not args.ensemble_only:
        # SAV, fixed step
        log("SAV fixed step")
        rs = [plan.sav_r(a), 0.0]
        rs[1] = rs[0]
        a2, b2 = a.clone(), b.clone()
        plan.run(a2, b2, scheme="sav", nsteps=20, k=k, k_prev=k, startup=False, rs=rs)
        torch.cuda.synchronize()
        ns = 200
        t0 = time.perf_counter()
        plan.run(a2, b2, scheme="sav", nsteps=ns, k=k, k_prev=k, startup=False, rs=rs)
        torch.cuda.synchronize()
        extra["sav_steps_per_s"] = round(ns / (time.perf_counter() - t0), 1)
        # adaptive IMEX (AM3 error control, sigma_tol 1e-5)
        log("adaptive IMEX")
        a2, b2 = uh0.clone(), torch.empty_like(uh0)
        opts = fch.AdaptOpts(sigma_tol=1e-5)
        plan.run(a2, b2, scheme="imex", adaptive=True, startup=True, t_end=1.0, nsteps=50,
                 adapt=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = plan.run(a2, b2, scheme="imex", adaptive=True, startup=True, t_end=10.0,
                        nsteps=300, adapt=opts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        extra["adaptive_imex_accepted_steps_per_s"] = round(info["accepted"] / el, 1)
        extra["adaptive_imex_attempts_per_s"] = round(
            (info["accepted"] + info["rejected"]) / el, 1)
        extra["adaptive_imex_mean_step"] = info["t"] / max(info["accepted"], 1)
        # adaptive SAV (the same control; r kept on the device)
        a2, b2 = uh0.clone(), torch.empty_like(uh0)
        plan.run(a2, b2, scheme="sav", adaptive=True, startup=True, t_end=1.0, nsteps=50,
                 adapt=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = plan.run(a2, b2, scheme="sav", adaptive=True, startup=True, t_end=10.0,
                        nsteps=300, adapt=opts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        extra["adaptive_sav_accepted_steps_per_s"] = round(info["accepted"] / el, 1)
        # ETDRK2 (Sec. 3.6): two chemical-potential evaluations (8 FFT calls,
        # 22 S of algorithmic traffic) per fixed step; adaptive attempts start
        # from the cached F(u^n) like IMEX's
        log("ETDRK2 fixed step and adaptive")
        a2, b2 = a.clone(), b.clone()
        plan.run(a2, b2, scheme="etd", nsteps=20, k=k)
        torch.cuda.synchronize()
        ne = 400
        t0 = time.perf_counter()
        plan.run(a2, b2, scheme="etd", nsteps=ne, k=k)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        extra["etd_steps_per_s"] = round(ne / el, 1)
        extra["etd_step_GBps"] = round(22 * S * ne / el / 1e9, 1)
        a2, b2 = uh0.clone(), torch.empty_like(uh0)
        plan.run(a2, b2, scheme="etd", adaptive=True, startup=True, t_end=1.0, nsteps=50,
                 adapt=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = plan.run(a2, b2, scheme="etd", adaptive=True, startup=True, t_end=10.0,
                        nsteps=300, adapt=opts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        extra["adaptive_etd_accepted_steps_per_s"] = round(info["accepted"] / el, 1)
        extra["adaptive_etd_attempts_per_s"] = round(
            (info["accepted"] + info["rejected"]) / el, 1)
        extra["adaptive_etd_mean_step"] = info["t"] / max(info["accepted"], 1)
        # the paper's cost measure: FFT calls to reach the same time at the same
        # local error target (sigma_tol 1e-5), from the same initial state
        log("FFT calls to t = 0.05, adaptive IMEX / SAV / ETDRK2")
        cost = {"t_end": 0.05, "sigma_tol": 1e-5}
        for sch in ("imex", "sav", "etd"):
            a2, b2 = uh0.clone(), torch.empty_like(uh0)
            plan.reset_stats()
            t0 = time.perf_counter()
            info = plan.run(a2, b2, scheme=sch, adaptive=True, startup=True, t_end=0.05,
                            nsteps=20000, adapt=opts)
            torch.cuda.synchronize()
            cost[sch] = {"accepted": info["accepted"], "rejected": info["rejected"],
                         "fft_calls": plan.stats()["fft_calls"],
                         "seconds": round(time.perf_counter() - t0, 3)}
        extra["fft_calls_to_t"] = cost
        # PSD (i_tol 1e-10, lambda from Table SearchSize)
        log("PSD")
        a2, b2 = a.clone(), b.clone()
        plan.reset_stats()
        t0 = time.perf_counter()
        npsd = 10
        info = plan.run(a2, b2, scheme="psd", nsteps=npsd, k=k, k_prev=k, startup=False,
                        psd_tol=1e-10)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        extra["psd_iterations_per_s"] = round(info["psd_iters"] / el, 1)
        extra["psd_fft_calls_per_step"] = round(4.0 * info["psd_iters"] / npsd, 2)
        extra["psd_steps_per_s"] = round(npsd / el, 1)
        c3, roofline_streaming = c3_leg(dev)
        extra["c3_psd_adaptive_2048"] = c3
        # 2D FFT bandwidth, streaming regime: R2C then C2R over a 32-field batch
        # (269 MB physical + 269 MB spectral + 269 MB staging, beyond the 256 MB
        # Infinity Cache), batched launches; and one field (cache-resident)
        fft_bytes = 8 * N * N + 3 * S      # per transform: P + 3S (one row<->column round trip)
        for B in (32, 1):
            log("FFT R2C + C2R, batch %d x 1024^2" % B)
            g = torch.Generator(device=dev)
            g.manual_seed(7)
            U = torch.randn((B, N, N), dtype=torch.float64, device=dev, generator=g)
            Uh = torch.empty((B, N // 2 + 1, N), dtype=torch.complex128, device=dev)
            ws = torch.empty(plan.lib_inverse_batch_ws_bytes(B), dtype=torch.uint8, device=dev)
            for _ in range(10):
                plan.forward_batch(U, out=Uh)
                plan.inverse_batch(Uh, out=U, ws=ws)
            iters = 20 if B > 1 else 400
            samples = []
            for _ in range(5):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(iters):
                    plan.forward_batch(U, out=Uh)
                    plan.inverse_batch(Uh, out=U, ws=ws)
                e1.record()
                e1.synchronize()
                samples.append(e0.elapsed_time(e1) * 1e-3 / (2 * B * iters))
            per_fft = sorted(samples)[2]
            extra["fft2d_batch%d" % B] = {
                "us_per_transform": round(per_fft * 1e6, 3),
                "GBps": round(fft_bytes / per_fft / 1e9, 1),
                "frac_of_8TBps": round(fft_bytes / per_fft / 8e12, 4),
                "bytes_per_transform": fft_bytes}
            del U, Uh, ws
    if not args.no_extra:
        # the critical-d sweep of Sec. 5.1 (Table f:defect-onsetR): 206 members of the
        # critical benchmark (256^2, the paper's initial data), adaptive IMEX at
        # sigma_tol 1e-5 to T = 250 in one batched ensemble
        if not args.ensemble_only:
            log("critical-d sweep: 206 members to T = 250")
            from paper_2006_04784_amd import sweeps
            sw = sweeps.critical_d_sweep(sweeps.paper_d_values(), sigma_tol=1e-5, t_end=250.0)
            extra["critical_d_sweep"] = {
                "scheme": "imex", "sigma_tol": 1e-5, "members": len(sw["d"]), "t_end": 250.0,
                "d_critical": sw["d_critical"],
                "d_max_without_defect": sw["d_max_without_defect"],
                "paper_d_critical_imex": 0.7540, "seconds": round(sw["seconds"], 2),
                "accepted_steps": int(sum(sw["accepted"])),
                "accepted_steps_per_s": round(sum(sw["accepted"]) / sw["seconds"], 1)}
        # batched ensemble: 64 adaptive IMEX runs of mixed size in captured graphs,
        # each capped at 2000 accepted steps; aggregate accepted steps/s over a
        # fixed wall window after warm-up, closed in chunks of 50 attempts while
        # every member is still running (no member reaches the cap inside it)
        log("ensemble of 64 mixed-size adaptive runs")
        mem = inputs.c4_members()
        ens_cap, window_s = 2000, 0.5
        ens = fch.Ensemble(mem, adapt=fch.AdaptOpts(sigma_tol=1e-5), t_end=1e9,
                           max_steps=ens_cap)
        for i, mi in enumerate(mem):
            ens.load(i, torch.from_numpy(inputs.c4_initial(mi, i)).to(dev))
        ens.autotune(reps=3)
        info = ens.run(max_attempts=20, sync_every=20, use_graph=True)     # warm-up attempts
        torch.cuda.synchronize()
        acc0, rej0, att = info["accepted"], info["rejected"], 0   # accepted/rejected: totals
        t0 = time.perf_counter()
        while True:
            info = ens.run(max_attempts=50, sync_every=50, use_graph=True)
            el = time.perf_counter() - t0     # run() returns after its final host wait
            att += info["attempts"]           # attempts: this call's
            if el >= window_s or info["active"] < len(mem):
                break
        extra["ensemble_accepted_steps_per_s"] = round((info["accepted"] - acc0) / el, 1)
        extra["ensemble"] = {"members": 64, "sizes": {str(n): sum(m["N"] == n for m in mem)
                                                      for n in (128, 256, 512, 1024)},
                             "cap_accepted_per_member": ens_cap, "window_s": round(el, 3),
                             "members_active_at_end": info["active"],
                             "accepted": info["accepted"] - acc0,
                             "rejected": info["rejected"] - rej0,
                             "attempts": att}
        ens.close()
        # the same ensemble machinery on 16 equal 1024^2 members: one batched
        # launch per stage covers all of them, so the row and column passes
        # overlap across members instead of draining per field
        log("ensemble of 16 adaptive 1024^2 runs")
        rng = np.random.default_rng(2025)
        mem = [dict(N=1024, L=1024 * 4 * np.pi / 256, eps=0.1,
                    eta1=float(rng.uniform(1.2, 1.6)), eta2=float(rng.uniform(1.5, 2.5)))
               for _ in range(16)]
        ens = fch.Ensemble(mem, adapt=fch.AdaptOpts(sigma_tol=1e-5), t_end=1e9, max_steps=320)
        for i, mi in enumerate(mem):
            ens.load(i, torch.from_numpy(inputs.circle_bilayer(
                1024, mi["L"], 0.1, seed=300 + i)).to(dev))
        ens.autotune(reps=3)
        ens.run(max_attempts=20, sync_every=20, use_graph=True)
        torch.cuda.synchronize()

        def member_attempts():
            rows = [ens.member(i, state=False, klog=False)[2] for i in range(len(mem))]
            return sum(r["accepted"] + r["rejected"] for r in rows)

        a0 = member_attempts()
        t0 = time.perf_counter()
        info = ens.run(max_attempts=100000, sync_every=100, use_graph=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        att = member_attempts() - a0
        S1024 = 16 * 1024 * 513
        extra["ensemble_1024x16"] = {
            "member_attempts_per_s": round(att / el, 1),
            "bytes_per_member_attempt": 26 * S1024,
            "GBps": round(26 * S1024 * att / el / 1e9, 1),
            "frac_of_8TBps": round(26 * S1024 * att / el / 8e12, 4),
            "member_attempts": att, "seconds": round(el, 3)}
        ens.close()
    if not args.no_extra and not args.ensemble_only:
        # learned PSD warm start at 256^2: PSD FFT calls per step, learned vs plain
        log("learned PSD warm start (data, training, held-out comparison)")
        from paper_2006_04784_amd import learned
        ev, _net, _plan = learned.run_experiment(range(16), [900, 901], nsteps=80, epochs=20,
                                                 batch=16, log=None, device=dev)
        ev.pop("per_step")
        extra["learned_warm_start"] = {k: (float("%.4g" % v) if isinstance(v, float) else v)
                                       for k, v in ev.items()}
        extra["learned_warm_start"]["scale"] = (
            "reduced: 16 training seeds x 80 accepted steps, 2 held-out seeds; the full "
            "configuration trains on 40 seeds x 500 steps (about 20k pairs)")
        extra["learned_warm_start"]["fft_calls_note"] = (
            "learned: 4 per PSD iteration plus the forward transform of the guess")
        # the same comparison at the workload's full scale: stored parameters
        # trained on about 20k pairs, held-out trajectories of 500 accepted steps
        log("learned PSD warm start, full scale (stored parameters, held-out 500-step runs)")
        evf = learned.evaluate_pretrained(learned.WEIGHTS_C5, [900, 901], nsteps=500,
                                          device=dev)
        evf.pop("per_step")
        extra["learned_warm_start_full_scale"] = {
            k: (float("%.4g" % v) if isinstance(v, float) else v) for k, v in evf.items()}
        extra["learned_warm_start_full_scale"]["scale"] = (
            "full: parameters trained on 40 seeds x 500 accepted steps (19960 pairs, 10 "
            "epochs; python -m paper_2006_04784_amd.learned --train-full), evaluated on "
            "held-out seeds 900 and 901, 500 accepted steps each")
    if args.copy_probe:
        # a plain elementwise copy of known size: 256 MiB read, 256 MiB written
        x = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)
        torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline (bounded sample)")
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        threads = max(1, min(threads, os.cpu_count() or 1))
        oracle.set_threads(threads)
        m = oracle.Model(**kw, zeta=plan.prm.zeta, D0=plan.prm.D0)
        un = oracle.r2c(u0)
        um = un.copy()
        n_done, t_cpu = 0, 0.0
        while t_cpu < 15.0 and n_done < 200:
            t0 = time.perf_counter()
            nxt = oracle.imex_step(m, un, um, k, k if n_done else -1.0)
            t_cpu += time.perf_counter() - t0
            um, un = un, nxt
            n_done += 1
        cpu = {"value": round(n_done / t_cpu, 4), "unit": "steps/s", "cores": threads,
               "kind": "oracle",
               "sample": "%d BDF2-IMEX steps of the 1024^2 workload (first is the startup "
                         "step), C oracle with OpenMP over FFT lines" % n_done}

    out = {
        "metric": "BDF2 steps/s and FFT HBM GB/s (FP64, 1024²); PSD FFT calls/step "
                  "learned vs plain",
        "value": round(steps_per_s, 2),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "m1: FCH 1024^2 on [0,16pi]^2, eps 0.1, eta (1.45, 2.0) eps, "
                               "q 0, fixed-step BDF2-IMEX k=1e-3, one circular bilayer r=0.3L",
                   "N": N, "scheme": "imex", "k": k,
                   "launch_config": dict(zip(("row_R", "row_E", "row_twl", "col_E", "col_twl"),
                                             plan.get_config())),
                   "autotuned": not args.config, "graph_steps": args.graph},
        "roofline": roofline,
        "roofline_streaming": roofline_streaming,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
