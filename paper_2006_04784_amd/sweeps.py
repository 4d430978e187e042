"""Studies of the paper's benchmarks on the GPU path: the critical background
level of defect onset (Sec. 5.1, Table f:defect-onsetR) as one batched
ensemble or by bisection, FFT calls against the stabilization beta
(Figure Find-Beta), fixed-step temporal convergence (Table tab:rates), the
schemes' final states compared (Table t:Comp-error) and grid refinement
(Table t:GRE).

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


def onset(ds, umax, threshold=DEFECT_THRESHOLD):
    """(smallest d whose running max of u crosses the threshold, largest d that
    does not), either None when there is no such d (Sec. 5.1 defect onset; a
    NaN maximum counts as no defect)."""
    over = [d for d, u in zip(ds, umax) if u > threshold]
    under = [d for d, u in zip(ds, umax) if not u > threshold]
    return (min(over) if over else None), (max(under) if under else None)


def critical_d_sweep(ds, sigma_tol=1e-5, t_end=250.0, t0=60.0, threshold=DEFECT_THRESHOLD,
                     N=256, physical_k=False, max_steps=1000000, device="cuda:0", log=None,
                     chunk=5000, scheme="imex", sampling="cell", n0=inputs.PAPER_N0):
    """Runs one ensemble member per d with one scheme (imex, sav or etd) and
    returns a dict with the per-member running max of u, accepted / rejected
    steps, end times, the critical d (None when no member crosses the
    threshold) and the wall time.  physical_k, sampling and n0 select a
    reading of the initial data (inputs.paper_initial_data)."""
    ds = [float(d) for d in ds]
    # d enters eq. dcoef as the constant eps d / alpha_m(0)^2 only: the filtered
    # strip is built once and shifted per member
    kw, base = inputs.paper_initial_data("critical", N=N, d=0.0, physical_k=physical_k,
                                         sampling=sampling, n0=n0)
    shift = kw["eps"] / inputs.PAPER_ALPHA0 ** 2
    members = [dict(kw) for _ in ds]
    u0s = [base + shift * d for d in ds]
    ens = fch.Ensemble(members, adapt=fch.AdaptOpts(sigma_tol=sigma_tol), t_end=t_end,
                       max_steps=max_steps, k_first=1e-9, device=device, umax_t0=t0,
                       scheme=scheme)
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
    d_crit, d_free = onset(ds, umax, threshold)
    if any(r["nonfinite"] for r in rows):
        raise RuntimeError("a member reached a non-finite state")
    if any(r["invalid"] for r in rows):
        raise RuntimeError("a SAV member reached E_1 + D_0 <= 0")
    return {"scheme": scheme, "d": ds, "umax": umax, "accepted": [r["accepted"] for r in rows],
            "rejected": [r["rejected"] for r in rows], "t": [r["t"] for r in rows],
            "d_critical": d_crit, "d_max_without_defect": d_free, "attempts": attempts,
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


def beta_sweep(scheme="sav", beta1s=(0.25, 0.5, 1.0, 1.5, 2.0, 2.5, 2.75), benchmarks=None,
               t_end=10.0, sigma_tol=1e-5, max_steps=200000, device="cuda:0", log=None):
    """FFT calls to reach t_end for the paper's benchmarks (Table t:Benchmark,
    their initial data) against the stabilization beta_1 of L_0 with
    beta_2 = 3 - beta_1 (Sec. 3.5, eq. e:SAV-L0), adaptive at sigma_tol.
    Runs that hit max_steps accepted steps are marked capped."""
    benchmarks = benchmarks or list(inputs.PAPER_BENCHMARKS)
    out = {}
    tw = time.perf_counter()
    for name in benchmarks:
        kw, u0 = inputs.paper_initial_data(name)
        rows = []
        for b1 in beta1s:
            plan = fch.Plan(**kw, beta1=b1, beta2=3.0 - b1, device=device)
            a = plan.forward(torch.from_numpy(np.ascontiguousarray(u0)).to(plan.device))
            b = torch.empty_like(a)
            plan.reset_stats()
            t1 = time.perf_counter()
            info = plan.run(a, b, scheme=scheme, adaptive=True, startup=True, t_end=t_end,
                            k_first=1e-9, nsteps=max_steps,
                            adapt=fch.AdaptOpts(sigma_tol=sigma_tol))
            row = {"beta1": b1, "beta2": 3.0 - b1, "fft_calls": plan.stats()["fft_calls"],
                   "accepted": info["accepted"], "rejected": info["rejected"],
                   "t": info["t"], "capped": info["t"] < t_end * (1 - 1e-12),
                   "seconds": round(time.perf_counter() - t1, 3)}
            rows.append(row)
            if log:
                log("%s %s beta1 %.2f: %d FFT calls, %d steps%s, %.1f s" %
                    (scheme, name, b1, row["fft_calls"], row["accepted"],
                     " (capped)" if row["capped"] else "", time.perf_counter() - tw))
            plan.close()
        out[name] = rows
    return out


def temporal_convergence(name="sub-critical", T=0.32, ks=None, schemes=("psd", "imex", "sav", "etd"),
                         ref_steps=1024, device="cuda:0"):
    """Fixed-step errors at time T from a benchmark's initial data against a
    fine BDF2-PSD reference (T / ref_steps, i_tol 1e-12), the comparison of
    Table tab:rates.  Returns {scheme: [relative L2 errors]} and the ks."""
    ks = list(ks or [0.08 / 2 ** j for j in range(7)])
    kw, u0 = inputs.paper_initial_data(name)
    plan = fch.Plan(**kw, device=device)
    uh0 = plan.forward(torch.from_numpy(np.ascontiguousarray(u0)).to(plan.device))

    def run(scheme, k, tol=1e-12):
        a, b = uh0.clone(), torch.empty_like(uh0)
        plan.run(a, b, scheme=scheme, nsteps=int(round(T / k)), k=k, psd_tol=tol,
                 psd_max_iter=5000, psd_lambda=1.0)
        return plan.inverse(a)

    ref = run("psd", T / ref_steps)
    nref = float(torch.linalg.norm(ref))
    out = {"T": T, "k": ks}
    for sch in schemes:
        out[sch] = [float(torch.linalg.norm(run(sch, k) - ref)) / nref for k in ks]
    return out


# Table tolPSD: the PSD tolerance ratio nu (i_tol = nu * sigma_tol, Sec. 3.3) and the
# optimal k_max per q
PSD_SETTINGS = {0.0: (1e-3, 0.05), 0.2: (2e-5, 0.02), 0.5: (1e-6, 0.01)}
# Table t:Comp-error: final time per benchmark
COMP_T = {"sub-critical": 250.0, "critical": 250.0, "super-critical": 250.0, "foot-1": 50.0,
          "foot-2": 50.0}


def scheme_comparison(benchmarks=None, sigma_tol=1e-5, schemes=("psd", "imex", "sav", "etd"),
                      device="cuda:0", log=None, max_steps=5000000):
    """Each scheme, adaptive at sigma_tol, from a benchmark's initial data to
    its final time of Table t:Comp-error (PSD with i_tol = nu sigma_tol and k_max
    of Table tolPSD; ETDRK2 only for the q = 0 benchmarks, as in the paper), and the
    relative L2 differences of the final states: the quantities of Table
    t:Comp-error.  Returns {benchmark: {"runs": {...}, "diff": {...}}}."""
    benchmarks = benchmarks or list(COMP_T)
    out = {}
    tw = time.perf_counter()
    for name in benchmarks:
        kw, u0 = inputs.paper_initial_data(name)
        plan = fch.Plan(**kw, device=device)
        uh0 = plan.forward(torch.from_numpy(np.ascontiguousarray(u0)).to(plan.device))
        nu, kmax = PSD_SETTINGS[kw["q"]]
        finals, runs = {}, {}
        for sch in schemes:
            if sch == "etd" and kw["q"] != 0.0:
                continue
            a, b = uh0.clone(), torch.empty_like(uh0)
            plan.reset_stats()
            t1 = time.perf_counter()
            try:
                info = plan.run(a, b, scheme=sch, adaptive=True, startup=True,
                                t_end=COMP_T[name], k_first=1e-9, nsteps=max_steps,
                                psd_tol=nu * sigma_tol,
                                psd_max_iter=20000,
                                adapt=fch.AdaptOpts(sigma_tol=sigma_tol,
                                                    k_max=kmax if sch == "psd" else float("inf")))
            except fch.FchError as ex:   # e.g. a PSD solve that missed its tolerance
                runs[sch] = {"error": str(ex)}
                if log:
                    log("%s %s: %s" % (name, sch, ex))
                continue
            finals[sch] = plan.inverse(a)
            runs[sch] = {"accepted": info["accepted"], "rejected": info["rejected"],
                         "t": info["t"], "fft_calls": plan.stats()["fft_calls"],
                         "psd_iters": info["psd_iters"], "max_u": float(finals[sch].max()),
                         "seconds": round(time.perf_counter() - t1, 2)}
            if log:
                log("%s %s: %d steps, %d FFT calls, max u %.3f, %.1f s" %
                    (name, sch, info["accepted"], runs[sch]["fft_calls"], runs[sch]["max_u"],
                     time.perf_counter() - tw))
        diff = {}
        pairs = [("imex", "psd"), ("sav", "psd"), ("sav", "imex"), ("etd", "psd")]
        for x, y in pairs:
            if x in finals and y in finals:
                diff["%s/%s" % (x, y)] = float(torch.linalg.norm(finals[x] - finals[y]) /
                                             torch.linalg.norm(finals[y]))
        out[name] = {"T": COMP_T[name], "runs": runs, "diff": diff}
        plan.close()
    return out


def grid_refinement(benchmarks=None, sigma_tol=1e-5, pairs=None, device="cuda:0", log=None):
    """Adaptive BDF2-PSD (i_tol = nu sigma_tol, k_max of Table tolPSD) from a
    benchmark's initial data at N and 2N to its final time of Table
    t:Comp-error; the absolute L2 difference h (sum over the N grid of
    (u_N - u_2N)^2)^(1/2), u_2N taken at the shared points: the quantity of
    Table t:GRE.  pairs: {benchmark: [(N, 2N), ...]}."""
    benchmarks = benchmarks or list(COMP_T)
    if pairs is None:
        pairs = {b: [(256, 512)] for b in benchmarks}
        if "foot-2" in pairs:     # the paper also refines foot-2 from 512 to 1024
            pairs["foot-2"] = [(256, 512), (512, 1024)]
    out = {}
    tw = time.perf_counter()
    cache = {}

    def final(name, N):
        if (name, N) in cache:
            return cache[(name, N)]
        kw, u0 = inputs.paper_initial_data(name, N=N)
        plan = fch.Plan(**kw, device=device)
        nu, kmax = PSD_SETTINGS[kw["q"]]
        a = plan.forward(torch.from_numpy(np.ascontiguousarray(u0)).to(plan.device))
        b = torch.empty_like(a)
        info = plan.run(a, b, scheme="psd", adaptive=True, startup=True, t_end=COMP_T[name],
                        k_first=1e-9, nsteps=5000000, psd_tol=nu * sigma_tol,
                        psd_max_iter=20000, adapt=fch.AdaptOpts(sigma_tol=sigma_tol, k_max=kmax))
        u = plan.inverse(a).cpu().numpy()
        plan.close()
        if log:
            log("%s N=%d: %d steps, %d PSD iterations, %.1f s" %
                (name, N, info["accepted"], info["psd_iters"], time.perf_counter() - tw))
        cache[(name, N)] = u
        return u

    for name in benchmarks:
        rows = []
        for (n1, n2) in pairs[name]:
            u1, u2 = final(name, n1), final(name, n2)
            h = inputs.PAPER_L / n1
            err = float(h * np.sqrt(np.sum((u1 - u2[::n2 // n1, ::n2 // n1]) ** 2)))
            rows.append({"N": n1, "N2": n2, "abs_l2": err})
        out[name] = rows
    return out


# ---- global error against cost ("dollars per digit", Sec. 5.2) ---------------
# local error targets of the sweep and the reference runs of Sec. 5.2: PSD at
# sigma_tol 1e-9 (q = 0) and 3e-8 (q = 0.2), IMEX at 3e-9 (q = 0.5)
DPD_SIGMAS = (1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7)
DPD_REFERENCE = {0.0: ("psd", 1e-9), 0.2: ("psd", 3e-8), 0.5: ("imex", 3e-9)}


def adaptive_final(plan, uh0, scheme, sigma_tol, t_end, q, max_steps=20000000, piece=20000,
                   log=None):
    """One adaptive run from uh0 to t_end at sigma_tol (PSD: i_tol = nu sigma_tol
    and k_max of Table tolPSD); returns (physical final state, run info with the
    FFT calls of the run).  The run proceeds in pieces of `piece` accepted
    steps, each continuing from the last two states and step sizes (and SAV's
    r history), which is the same trajectory as one call; log reports each."""
    nu, kmax = PSD_SETTINGS[q]
    a, b = uh0.clone(), torch.empty_like(uh0)
    plan.reset_stats()
    t1 = time.perf_counter()
    opts = fch.AdaptOpts(sigma_tol=sigma_tol, k_max=kmax if scheme == "psd" else float("inf"))
    tot = {"accepted": 0, "rejected": 0, "psd_iters": 0}
    t, info, rs = 0.0, None, None
    while t < t_end * (1 - 1e-14) and tot["accepted"] < max_steps:
        n = min(piece, max_steps - tot["accepted"])
        if info is None:
            info = plan.run(a, b, scheme=scheme, adaptive=True, startup=True, t_end=t_end,
                            k_first=1e-9, nsteps=n, psd_tol=nu * sigma_tol, psd_max_iter=20000,
                            adapt=opts)
        else:
            info = plan.run(a, b, scheme=scheme, adaptive=True, startup=False, t_end=t_end - t,
                            k=info["k_next"], k_prev=info["k_last"], nsteps=n, rs=rs,
                            psd_tol=nu * sigma_tol, psd_max_iter=20000, adapt=opts)
        rs = info["rs"]
        t += info["t"]
        for key in tot:
            tot[key] += info[key]
        if log and t < t_end * (1 - 1e-14):
            log("  %s sigma %.0e: t = %.4g after %d steps" % (scheme, sigma_tol, t, tot["accepted"]))
    info = dict(info, t=t, **tot)
    info["fft_calls"] = plan.stats()["fft_calls"]
    info["seconds"] = round(time.perf_counter() - t1, 2)
    return plan.inverse(a), info


def cost_at_error(rows, target):
    """FFT calls at which each scheme's global error first falls to target, going
    down its sigma_tol sweep: log-log interpolation between the last run above
    and the first at or below the target (None if no run reaches it; the first
    run's calls, flagged, if the coarsest already does).  Also the fewest FFT
    calls of any run at or below the target ("cheapest_run"), which differs
    where the cost does not grow monotonically down the sweep."""
    out = {}
    for sch in sorted({r["scheme"] for r in rows}):
        rs = sorted([r for r in rows if r["scheme"] == sch and "error" in r],
                    key=lambda r: -r["sigma_tol"])
        ok = [r for r in rs if r["error"] <= target]
        cheapest = min(ok, key=lambda r: r["fft_calls"]) if ok else None
        hit = None
        for i, r in enumerate(rs):
            if r["error"] <= target:
                if i == 0:
                    hit = {"fft_calls": r["fft_calls"], "sigma_tol": r["sigma_tol"],
                           "coarsest_run": True}
                else:
                    p = rs[i - 1]
                    w = (np.log(target) - np.log(p["error"])) / (np.log(r["error"]) -
                                                                  np.log(p["error"]))
                    calls = np.exp(np.log(p["fft_calls"]) +
                                   w * (np.log(r["fft_calls"]) - np.log(p["fft_calls"])))
                    hit = {"fft_calls": float(calls),
                           "between_sigma_tol": (p["sigma_tol"], r["sigma_tol"])}
                break
        if hit is not None:
            hit["cheapest_run"] = {"fft_calls": cheapest["fft_calls"],
                                   "sigma_tol": cheapest["sigma_tol"]}
        out[sch] = hit
    return out


def cost_vs_error(name="super-critical", sigmas=DPD_SIGMAS, schemes=("imex", "sav", "psd", "etd"),
                  reference=None, etd_min_sigma=1e-6, psd_sigmas=None, device="cuda:0",
                  log=None, targets=(2.5e-3, 7e-4)):
    """Global relative L2 error at the benchmark's final time (Table
    t:Comp-error) against the total FFT calls of each scheme over a sweep of
    sigma_tol, measured against the reference run of Sec. 5.2 (DPD_REFERENCE;
    ETDRK2 only for q = 0, as in the paper).  Returns the runs and, per target
    error, each scheme's interpolated FFT calls (cost_at_error)."""
    kw, u0 = inputs.paper_initial_data(name)
    q = kw["q"]
    T = COMP_T[name]
    plan = fch.Plan(**kw, device=device)
    uh0 = plan.forward(torch.from_numpy(np.ascontiguousarray(u0)).to(plan.device))
    ref_scheme, ref_sigma = reference or DPD_REFERENCE[q]
    tw = time.perf_counter()
    try:
        u_ref, info = adaptive_final(plan, uh0, ref_scheme, ref_sigma, T, q, log=log)
    except fch.FchError as ex:
        # the reference of Sec. 5.2 did not finish (a PSD solve missed its
        # tolerance); the q = 0.5 reference (IMEX at 3e-9) stands in
        if log:
            log("%s reference %s sigma %.0e failed (%s); IMEX at 3e-9 instead" %
                (name, ref_scheme, ref_sigma, ex))
        ref_scheme, ref_sigma = "imex", 3e-9
        u_ref, info = adaptive_final(plan, uh0, ref_scheme, ref_sigma, T, q, log=log)
    nref = float(torch.linalg.norm(u_ref))
    if log:
        log("%s reference %s sigma %.0e: %d steps, %d FFT calls, %.1f s" %
            (name, ref_scheme, ref_sigma, info["accepted"], info["fft_calls"],
             time.perf_counter() - tw))
    rows = []
    for sch in schemes:
        if sch == "etd" and q != 0.0:
            continue
        for sg in (psd_sigmas if sch == "psd" and psd_sigmas else sigmas):
            if sch == "etd" and sg < etd_min_sigma:
                continue
            row = {"scheme": sch, "sigma_tol": sg}
            try:
                u, inf_ = adaptive_final(plan, uh0, sch, sg, T, q, log=log)
                row.update(error=float(torch.linalg.norm(u - u_ref)) / nref,
                           fft_calls=int(inf_["fft_calls"]), accepted=int(inf_["accepted"]),
                           rejected=int(inf_["rejected"]), psd_iters=int(inf_["psd_iters"]),
                           seconds=inf_["seconds"])
            except fch.FchError as ex:   # e.g. a PSD solve that missed its tolerance
                row["failed"] = str(ex)
            rows.append(row)
            if log:
                log("%s %s sigma %.0e: %s (%.1f s)" % (
                    name, sch, sg, {k: row[k] for k in ("error", "fft_calls", "accepted")
                                    if k in row} or row.get("failed"),
                    time.perf_counter() - tw))
    plan.close()
    return {"benchmark": name, "T": T, "N": kw["N"], "q": q,
            "reference": {"scheme": ref_scheme, "sigma_tol": ref_sigma,
                          "accepted": int(info["accepted"]), "fft_calls": int(info["fft_calls"])},
            "runs": rows, "cost_at": {str(t): cost_at_error(rows, t) for t in targets}}


def psd_iteration_readings(name="foot-1", sigma_tol=1e-5, factors=(1.0, 10.0, 100.0),
                           lambdas=(), device="cuda:0", log=None):
    """Total PSD iterations of the adaptive run to the benchmark's final time
    (Table t:Comp-error) for stopping tolerances i_tol = f nu sigma_tol (nu and
    k_max of Table tolPSD): the quantity of Table tolPSD under readings of the
    tolerance.  Each lambda in `lambdas` adds a run at f = 1 with that fixed
    step length of eq. recurrence in place of Table SearchSize's."""
    kw, u0 = inputs.paper_initial_data(name)
    q = kw["q"]
    nu, kmax = PSD_SETTINGS[q]
    plan = fch.Plan(**kw, device=device)
    uh0 = plan.forward(torch.from_numpy(np.ascontiguousarray(u0)).to(plan.device))
    out = []
    for f, lam in [(f, 0.0) for f in factors] + [(1.0, lam) for lam in lambdas]:
        a, b = uh0.clone(), torch.empty_like(uh0)
        plan.reset_stats()
        t1 = time.perf_counter()
        row = {"benchmark": name, "sigma_tol": sigma_tol, "i_tol": f * nu * sigma_tol,
               "lambda": lam if lam > 0 else "Table SearchSize"}
        try:
            info = plan.run(a, b, scheme="psd", adaptive=True, startup=True, t_end=COMP_T[name],
                            k_first=1e-9, nsteps=5000000, psd_tol=f * nu * sigma_tol,
                            psd_max_iter=20000, psd_lambda=lam,
                            adapt=fch.AdaptOpts(sigma_tol=sigma_tol, k_max=kmax))
            row.update(psd_iters=int(info["psd_iters"]), accepted=int(info["accepted"]),
                       rejected=int(info["rejected"]))
        except fch.FchError as ex:
            row["failed"] = str(ex)
        row["seconds"] = round(time.perf_counter() - t1, 1)
        out.append(row)
        if log:
            log(str(row))
    plan.close()
    return out


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
                    help="ensemble-imex / ensemble-sav / ensemble-etd (all d at once) or "
                         "imex / sav / psd / etd (bisection with single runs)")
    ap.add_argument("--psd-nu", type=float, default=1e-3,
                    help="PSD stopping tolerance i_tol = nu * sigma (Table tolPSD: 1e-3 at q = 0)")
    ap.add_argument("--k-max", type=float, default=float("inf"))
    ap.add_argument("--beta-sweep", action="store_true",
                    help="FFT calls to --t-end against beta_1 (beta_2 = 3 - beta_1) instead")
    ap.add_argument("--max-steps", type=int, default=50000)
    ap.add_argument("--benchmarks", default="", help="comma-separated subset for --gre")
    ap.add_argument("--gre", action="store_true",
                    help="PSD grid refinement errors N vs 2N (Table t:GRE) instead")
    ap.add_argument("--compare", action="store_true",
                    help="all schemes on the five benchmarks to their final times instead")
    ap.add_argument("--rates", action="store_true",
                    help="fixed-step errors at T = 0.32 against a fine PSD reference instead")
    ap.add_argument("--cost", default="",
                    help="global error against FFT calls over a sigma_tol sweep (Sec. 5.2) for "
                         "the named benchmark instead")
    ap.add_argument("--sigmas", default="", help="comma-separated sigma_tol values for --cost")
    ap.add_argument("--psd-sigmas", default="", help="sigma_tol values of PSD for --cost")
    ap.add_argument("--schemes", default="imex,sav,psd,etd", help="schemes for --cost")
    ap.add_argument("--readings", action="store_true",
                    help="critical d of each initial-data reading (filter wavenumbers, sampling "
                         "of the strip, its mesh) at each --sigmas value instead")
    ap.add_argument("--psd-readings", default="",
                    help="PSD iterations to the final time of the named benchmark for i_tol = "
                         "f nu sigma_tol, f = 1, 10, 100, instead")
    ap.add_argument("--psd-lambdas", default="",
                    help="fixed PSD step lengths to add to --psd-readings (comma-separated)")
    args = ap.parse_args()
    if args.psd_readings:
        lams = tuple(float(x) for x in args.psd_lambdas.split(",")) if args.psd_lambdas else ()
        print(json.dumps(psd_iteration_readings(args.psd_readings, sigma_tol=args.sigma,
                                                lambdas=lams,
                                                log=lambda m: print(m, file=sys.stderr,
                                                                    flush=True))))
        sys.exit(0)
    if args.readings:
        sig = tuple(float(x) for x in args.sigmas.split(",")) if args.sigmas else (1e-5, 1e-6, 1e-7)
        err = lambda m: print(m, file=sys.stderr, flush=True)
        readings = {"cell-average, integer k": {}, "point sampling": {"sampling": "point"},
                    "512 indicator mesh": {"n0": 512}, "physical k": {"physical_k": True}}
        out = []
        for label, kwr in readings.items():
            for sg in sig:
                r = critical_d_sweep(paper_d_values(), sigma_tol=sg, t_end=args.t_end, t0=args.t0,
                                     log=err, **kwr)
                row = {"reading": label, "sigma_tol": sg, "d_critical": r["d_critical"],
                       "d_max_without_defect": r["d_max_without_defect"],
                       "umax_range_no_defect": max([u for u in r["umax"] if not u > DEFECT_THRESHOLD],
                                                   default=None),
                       "umax_min_defect": min([u for u in r["umax"] if u > DEFECT_THRESHOLD],
                                              default=None),
                       "seconds": round(r["seconds"], 1)}
                err(json.dumps(row))
                out.append(row)
        print(json.dumps(out))
        sys.exit(0)
    if args.cost:
        sig = tuple(float(x) for x in args.sigmas.split(",")) if args.sigmas else DPD_SIGMAS
        psig = tuple(float(x) for x in args.psd_sigmas.split(",")) if args.psd_sigmas else None
        print(json.dumps(cost_vs_error(args.cost, sigmas=sig, schemes=tuple(args.schemes.split(",")),
                                       psd_sigmas=psig,
                                       log=lambda m: print(m, file=sys.stderr, flush=True))))
        sys.exit(0)
    if args.rates:
        print(json.dumps(temporal_convergence()))
        sys.exit(0)
    if args.gre:
        print(json.dumps(grid_refinement(args.benchmarks.split(",") if args.benchmarks else None,
                                         log=lambda m: print(m, file=sys.stderr, flush=True))))
        sys.exit(0)
    if args.compare:
        print(json.dumps(scheme_comparison(sigma_tol=args.sigma,
                                           log=lambda m: print(m, file=sys.stderr, flush=True))))
        sys.exit(0)
    if args.beta_sweep:
        sch = "sav" if args.scheme.startswith("ensemble-") else args.scheme
        print(json.dumps(beta_sweep(sch, t_end=args.t_end, sigma_tol=args.sigma,
                                    max_steps=args.max_steps,
                                    log=lambda m: print(m, file=sys.stderr, flush=True))))
        sys.exit(0)
    ds = [d for d in paper_d_values()
          if (args.d_min is None or d >= args.d_min) and (args.d_max is None or d <= args.d_max)]
    err = lambda m: print(m, file=sys.stderr, flush=True)
    if args.scheme.startswith("ensemble-"):
        res = critical_d_sweep(ds, sigma_tol=args.sigma, t_end=args.t_end, t0=args.t0, log=err,
                               scheme=args.scheme[len("ensemble-"):])
        res["sigma_tol"] = args.sigma
    else:
        res = critical_d_bisect(args.scheme, args.sigma, ds, log=err, t_end=args.t_end,
                                t0=args.t0, k_max=args.k_max, psd_tol=args.psd_nu * args.sigma)
    print(json.dumps(res))
