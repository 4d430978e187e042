"""Timing of the CPU oracle (test infrastructure, not collected by pytest).

Fixed-step BDF2-IMEX steps/s at several grid sizes and BDF2-PSD iterations/s,
each with one thread and with all the threads OpenMP is given, on the
circle workload of each size (eps 0.1, L = N 4 pi / 256).  Each measurement
runs steps until about `budget` seconds have passed and reports the median of
`reps` such runs.  Usage: python tests/oracle_timing.py [--budget S] [--reps R]
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--budget", type=float, default=2.0)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
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
