"""Critical background level of defect onset (Sec. 5.1, Table f:defect-onsetR)
as one batched ensemble.

The critical benchmark of Table t:Benchmark is run for a range of the
initial-data parameter d (eq. dcoef), one ensemble member per value, with
adaptive BDF2-IMEX at a given local error target.  A bilayer's profile peaks
near u = 0.36 while defects sit deeper in the right well (u near 0.74), so
the running maximum of u over the accepted states after the initial
relaxation (t >= t0; early on every member's maximum overshoots to about 0.9
while the smoothed strip sharpens into a bilayer) separates the two outcomes.
The critical d is the smallest value whose maximum crosses a threshold
between them.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import fch, inputs

DEFECT_THRESHOLD = 0.55   # between the bilayer's peak (0.3566) and a defect's (about 0.74)


def critical_d_sweep(ds, sigma_tol=1e-5, t_end=250.0, t0=60.0, threshold=DEFECT_THRESHOLD,
                     N=256, physical_k=False, max_steps=1000000, device="cuda:0", log=None,
                     chunk=5000):
    """Runs one member per d and returns a dict with the per-member running
    max of u, accepted / rejected steps, end times, the critical d (None when
    no member crosses the threshold) and the wall time."""
    ds = [float(d) for d in ds]
    members, u0s = [], []
    for d in ds:
        kw, u0 = inputs.paper_initial_data("critical", N=N, d=d, physical_k=physical_k)
        members.append(kw)
        u0s.append(u0)
    ens = fch.Ensemble(members, adapt=fch.AdaptOpts(sigma_tol=sigma_tol), t_end=t_end,
                       max_steps=max_steps, k_first=1e-9, device=device, umax_t0=t0)
    for i, u0 in enumerate(u0s):
        ens.load(i, torch.from_numpy(np.ascontiguousarray(u0)).to(device))
    ens.autotune(5)
    tw = time.perf_counter()
    attempts = 0
    while True:
        info = ens.run(max_attempts=chunk, sync_every=250)
        attempts += info["attempts"]
        if log:
            log("d-sweep: %d attempts, %d members active, %.1f s" %
                (attempts, info["active"], time.perf_counter() - tw))
        if info["active"] == 0:
            break
    wall = time.perf_counter() - tw
    rows = [ens.member(i, state=False, klog=False)[2] for i in range(len(ds))]
    umax = [r["umax"] for r in rows]
    over = [d for d, u in zip(ds, umax) if u > threshold]
    under = [d for d, u in zip(ds, umax) if not u > threshold]
    if any(r["nonfinite"] for r in rows):
        raise RuntimeError("a member reached a non-finite state")
    return {"d": ds, "umax": umax, "accepted": [r["accepted"] for r in rows],
            "rejected": [r["rejected"] for r in rows], "t": [r["t"] for r in rows],
            "d_critical": min(over) if over else None,
            "d_max_without_defect": max(under) if under else None, "attempts": attempts,
            "seconds": wall}


def defect_onset_single(plan, d, scheme, sigma_tol, t_end=250.0, t0=60.0, dt_check=10.0,
                        k_max=float("inf"), psd_tol=1e-10, physical_k=False):
    """One adaptive run of the critical benchmark at background level d with a
    single plan (any scheme of fch_run): the largest u at the checkpoints
    t0, t0 + dt_check, ..., t_end (each segment ends exactly on its checkpoint,
    then the run continues from the last accepted step and trial step).
    Returns (max u over the checkpoints, accepted steps, FFT calls)."""
    kw, u0 = inputs.paper_initial_data("critical", N=plan.N, d=d, physical_k=physical_k)
    a = plan.forward(torch.from_numpy(np.ascontiguousarray(u0)).to(plan.device))
    b = torch.empty_like(a)
    opts = fch.AdaptOpts(sigma_tol=sigma_tol, k_max=k_max)
    plan.reset_stats()
    info = plan.run(a, b, scheme=scheme, adaptive=True, startup=True, t_end=t0, k_first=1e-9,
                    adapt=opts, psd_tol=psd_tol, psd_max_iter=20000)
    accepted = info["accepted"]
    um = float(plan.inverse(a).max())
    t = info["t"]
    while t < t_end * (1 - 1e-12):
        nxt = min(t + dt_check, t_end)
        info = plan.run(a, b, scheme=scheme, adaptive=True, startup=False, t_end=nxt - t,
                        k=info["k_next"], k_prev=info["k_last"], adapt=opts, psd_tol=psd_tol,
                        psd_max_iter=20000, rs=info["rs"])
        accepted += info["accepted"]
        t = nxt
        um = max(um, float(plan.inverse(a).max()))
    return um, accepted, plan.stats()["fft_calls"]


def critical_d_bisect(scheme, sigma_tol, ds=None, threshold=DEFECT_THRESHOLD, log=None,
                      device="cuda:0", **kw):
    """Bisection over the sorted d values for the smallest one with a defect
    (assuming the outcome is monotone in d), one single-plan run per probe.
    Returns a dict with the critical d, the probes and the wall time."""
    ds = sorted(ds or paper_d_values())
    b = inputs.PAPER_BENCHMARKS["critical"]
    plan = fch.Plan(N=256, L=inputs.PAPER_L, eps=0.1, eta1=b["eta1"], eta2=b["eta2"], q=b["q"],
                    device=device)
    probes = {}
    tw = time.perf_counter()

    def defect(i):
        um, acc, ffts = defect_onset_single(plan, ds[i], scheme, sigma_tol, **kw)
        probes[ds[i]] = {"umax": um, "accepted": acc, "fft_calls": ffts}
        if log:
            log("%s sigma %g d %.4f: max u %.4f, %d steps, %d FFT calls, %.1f s" %
                (scheme, sigma_tol, ds[i], um, acc, ffts, time.perf_counter() - tw))
        return um > threshold

    lo, hi = 0, len(ds) - 1
    if defect(lo):
        crit = ds[lo]
    elif not defect(hi):
        crit = None
    else:
        while hi - lo > 1:        # ds[lo] has no defect, ds[hi] has one
            mid = (lo + hi) // 2
            if defect(mid):
                hi = mid
            else:
                lo = mid
        crit = ds[hi]
    return {"scheme": scheme, "sigma_tol": sigma_tol, "d_critical": crit, "probes": probes,
            "seconds": time.perf_counter() - tw}


def paper_d_values():
    """The paper's sweep: d = 0.7523, 0.7524, ..., 0.7728."""
    return [round(0.7523 + 1e-4 * i, 4) for i in range(206)]


if __name__ == "__main__":
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--sigma", type=float, default=1e-5)
    ap.add_argument("--t-end", type=float, default=250.0)
    ap.add_argument("--t0", type=float, default=60.0)
    ap.add_argument("--d-min", type=float, default=None)
    ap.add_argument("--d-max", type=float, default=None)
    ap.add_argument("--scheme", default="ensemble-imex",
                    help="ensemble-imex (all d at once) or imex / sav / psd / etd (bisection)")
    ap.add_argument("--psd-tol", type=float, default=1e-3)
    ap.add_argument("--k-max", type=float, default=float("inf"))
    args = ap.parse_args()
    ds = [d for d in paper_d_values()
          if (args.d_min is None or d >= args.d_min) and (args.d_max is None or d <= args.d_max)]
    err = lambda m: print(m, file=sys.stderr, flush=True)
    if args.scheme == "ensemble-imex":
        res = critical_d_sweep(ds, sigma_tol=args.sigma, t_end=args.t_end, t0=args.t0, log=err)
        res["sigma_tol"] = args.sigma
    else:
        res = critical_d_bisect(args.scheme, args.sigma, ds, log=err, t_end=args.t_end,
                                t0=args.t0, k_max=args.k_max, psd_tol=args.psd_tol)
    print(json.dumps(res))
