"""Timing of the CPU oracle (test infrastructure, not collected by pytest).

Fixed-step BDF2-IMEX steps/s at several grid sizes and BDF2-PSD iterations/s,
each with one thread and with all the threads OpenMP is given, on the
circle workload of each size (eps 0.1, L = N 4 pi / 256).  Each measurement
runs steps until about `budget` seconds have passed and reports the median of
`reps` such runs.  With --workloads it times whole runs instead, with all
threads: the 200-step 64^2 IMEX run, adaptive IMEX on the 512^2 workload to
T = 10 (sigma_tol 1e-5) and the first 10 accepted adaptive PSD steps of the
2048^2 workload (sigma_tol 1e-6, k_max 0.05, i_tol 1e-10), each driven by the
oracle's steppers and its Sec. 3.2 controller.
Usage: python tests/oracle_timing.py [--budget S] [--reps R] [--workloads]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
from paper_2006_04784_amd import inputs  # noqa: E402


def _model(N):
    L = N * 4 * np.pi / 256
    return oracle.Model(N=N, L=L, eps=0.1, eta1=1.45, eta2=2.0, zeta=1.1, D0=L * L * 1.05), \
        oracle.r2c(inputs.circle_bilayer(N, L, 0.1, seed=0))


def imex_rate(N, threads, budget):
    oracle.set_threads(threads)
    m, uh0 = _model(N)
    um, un = uh0, oracle.imex_step(m, uh0, None, 1e-3, -1.0)
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget or n < 1:
        um, un = un, oracle.imex_step(m, un, um, 1e-3, 1e-3)
        n += 1
    return n / (time.perf_counter() - t0)


def psd_rate(N, threads, budget):
    oracle.set_threads(threads)
    m, uh0 = _model(N)
    u1 = oracle.imex_step(m, uh0, None, 1e-3, -1.0)
    its, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget or its < 1:
        _, it, _, _ = oracle.psd_step(m, u1, uh0, 1e-3, 1e-3, fixed_iters=4, lam=1.34)
        its += it
    return its / (time.perf_counter() - t0)


def adaptive_run(m, uh0, scheme, t_end, sigma_tol, k_max=float("inf"), k_first=1e-9,
                 max_accepted=None, psd_tol=1e-10):
    """Sec. 3.2 with the oracle: a first-order startup step of k_first, then
    attempts checked by the AM3 estimate; returns (accepted, rejected, t)."""
    step = (lambda un, um, k, kn: oracle.imex_step(m, un, um, k, kn)) if scheme == "imex" else \
        (lambda un, um, k, kn: oracle.psd_step(m, un, um, k, kn, tol=psd_tol, max_iter=20000)[0])
    prev = oracle.r2c(uh0) if uh0.ndim == 2 and not np.iscomplexobj(uh0) else uh0
    cur = step(prev, None, k_first, -1.0)
    Fm, Fn = oracle.F(m, prev), oracle.F(m, cur)
    t, kn, kt = k_first, k_first, k_first
    acc_n, rej_n = 1, 0
    while t < t_end * (1 - 1e-14) and (max_accepted is None or acc_n < max_accepted):
        kt = min(kt, t_end - t)
        trial = step(cur, prev, kt, kn)
        Ft = oracle.F(m, trial)
        e = oracle.am3_error(m, trial, cur, Ft, Fn, Fm, kt, kn)
        ok, knext = oracle.adapt_decide(e, kt, sigma_tol, 1e-9, k_max)
        if ok:
            prev, cur, Fm, Fn = cur, trial, Fn, Ft
            t, kn = t + kt, kt
            acc_n += 1
            if acc_n % 250 == 0:
                print("  %s: %d accepted, t = %.4g" % (scheme, acc_n, t), flush=True)
        else:
            rej_n += 1
        kt = knext
    return acc_n, rej_n, t


def workloads(threads):
    oracle.set_threads(threads)
    out = {}
    kw, u0 = inputs.workload("c1")
    m = oracle.Model(**kw)
    t0 = time.perf_counter()
    oracle.run_fixed(m, "imex", oracle.r2c(u0), 1e-3, 200)
    out["c1_200_imex_steps_s"] = round(time.perf_counter() - t0, 3)
    print("c1", out["c1_200_imex_steps_s"], flush=True)
    kw, u0 = inputs.workload("c2")
    m = oracle.Model(**kw)
    t0 = time.perf_counter()
    a, r, t = adaptive_run(m, u0, "imex", 10.0, 1e-5)
    out["c2_adaptive_imex_to_T10"] = {"seconds": round(time.perf_counter() - t0, 1),
                                      "accepted": a, "rejected": r, "t": t}
    print("c2", out["c2_adaptive_imex_to_T10"], flush=True)
    kw, u0 = inputs.workload("c3")
    m = oracle.Model(**kw)
    t0 = time.perf_counter()
    a, r, t = adaptive_run(m, u0, "psd", 1e9, 1e-6, k_max=0.05, max_accepted=11)
    out["c3_first_10_psd_steps"] = {"seconds": round(time.perf_counter() - t0, 1),
                                    "accepted_after_startup": a - 1, "rejected": r, "t": t}
    print("c3", out["c3_first_10_psd_steps"], flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--budget", type=float, default=2.0)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--workloads", action="store_true")
    args = ap.parse_args()
    if args.workloads:
        allt = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        print(json.dumps({"threads": allt, **workloads(allt)}))
        return
    allt = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"threads_all": allt, "cpu": os.cpu_count(), "imex_steps_per_s": {},
           "psd_iterations_per_s": {}}
    for N in (64, 512, 1024, 2048):
        out["imex_steps_per_s"][N] = {
            str(th): float(np.median([imex_rate(N, th, args.budget) for _ in range(args.reps)]))
            for th in (1, allt)}
        print("imex", N, out["imex_steps_per_s"][N], flush=True)
    for N in (256, 2048):
        out["psd_iterations_per_s"][N] = {
            str(th): float(np.median([psd_rate(N, th, args.budget) for _ in range(args.reps)]))
            for th in (1, allt)}
        print("psd", N, out["psd_iterations_per_s"][N], flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
