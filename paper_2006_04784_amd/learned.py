"""Learned PSD warm start: data generation with the library's adaptive
BDF2-PSD solver, training of :class:`nn.WarmStartNet` on the GPU, and the
comparison of PSD iteration counts (and FFT calls) from the learned guess
against the extrapolated guess of eq. recurrence at the same stopping
tolerance.  Orchestration only: the solves, transforms and network passes
run in the library's kernels.
"""
from __future__ import annotations

import os
import time

import numpy as np
import torch

from . import fch, inputs
from .nn import WarmStartNet


def c5_model(seed_eps=0.05):
    """Model parameters of the 256^2 warm-start workload ([0, 4 pi]^2, eps 0.05)."""
    return dict(N=256, L=4 * np.pi, eps=seed_eps, eta1=1.45, eta2=2.0)


def c5_initial(seed):
    kw = c5_model()
    return inputs.perturbed_circles(kw["N"], kw["L"], kw["eps"], 3, seed=seed,
                                    r_range=(0.5, 1.5))


def psd_trajectory(plan, u0, nsteps, sigma_tol=1e-5, k_max=0.05, tol=1e-10, k_first=1e-6,
                   max_iter=2000, t_burn=0.0):
    """Adaptive BDF2-PSD run (Sec. 3.2 step control, Sec. 3.3 solver) from the
    physical state u0 (numpy).  Returns the accepted physical states
    (torch float64, (nsteps+1, N, N)) and step sizes (numpy, k[i] = t_i - t_{i-1}).
    A solve that does not reach the tolerance within max_iter iterations (at
    the largest steps of this stiff workload) counts as a rejected attempt
    and halves the trial step.  t_burn > 0: the run first advances to
    t = t_burn under device control (fch_run) and records from there, so
    the recorded steps are the large, iteration-heavy steps of the later run
    rather than the startup transient."""
    dev = plan.device
    opts = fch.AdaptOpts(sigma_tol=sigma_tol, k_max=k_max)
    cur = plan.forward(torch.from_numpy(u0).to(dev))
    if t_burn > 0:
        prev = torch.empty_like(cur)
        info = plan.run(cur, prev, scheme="psd", adaptive=True, startup=True, k_first=k_first,
                        t_end=t_burn, adapt=opts, psd_tol=tol, psd_max_iter=max_iter)
        states = [plan.inverse(prev), plan.inverse(cur)]
        kn, kt = info["k_last"], info["k_next"]
        ks = [0.0, kn]
    else:
        states = [plan.inverse(cur)]
        prev, st = plan.step_psd(cur, None, k_first, -1.0, tol=tol)
        cur, prev = prev, cur
        states.append(plan.inverse(cur))
        ks = [0.0, k_first]
        kn, kt = k_first, k_first
    Fn, Fm = plan.rhs(cur), plan.rhs(prev)
    attempts = 0
    while len(states) <= nsteps and attempts < 20 * nsteps:
        attempts += 1
        trial, st = plan.step_psd(cur, prev, kt, kn, tol=tol, max_iter=max_iter,
                                  raise_noconv=False)
        if st["status"] == fch.FCH_E_NOCONV:
            kt *= 0.5
            continue
        Ft, acc, knext, err = plan.adapt_dt(trial, cur, Fn, Fm, kt, kn, opts)
        if acc:
            prev, cur = cur, trial
            Fm, Fn = Fn, Ft
            kn = kt
            ks.append(kt)
            states.append(plan.inverse(cur))
        kt = knext
    return torch.stack(states), np.array(ks)


def make_pairs(trajs):
    """(u^{n-1}, u^n, u^{n+1}, (k_{n+1}, k_n)) for n >= 1 of each trajectory."""
    idx = []
    for t, (S, ks) in enumerate(trajs):
        for n in range(1, S.shape[0] - 1):
            idx.append((t, n, ks[n + 1], ks[n]))
    return idx


def gather(trajs, items, dev):
    un = torch.stack([trajs[t][0][n] for t, n, _, _ in items])
    um = torch.stack([trajs[t][0][n - 1] for t, n, _, _ in items])
    up = torch.stack([trajs[t][0][n + 1] for t, n, _, _ in items])
    k = torch.tensor([[k1, k0] for _, _, k1, k0 in items], dtype=torch.float64, device=dev)
    return un, um, up, k


def train(net: WarmStartNet, trajs, epochs=20, lr=1e-3, seed=0, log=None):
    """Mini-batch Adam on the MSE of the normalized correction."""
    pairs = make_pairs(trajs)
    rng = np.random.default_rng(seed)
    losses = []
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        tot, nb_tot = 0.0, 0
        for s in range(0, len(order) - net.B + 1, net.B):
            items = [pairs[i] for i in order[s:s + net.B]]
            un, um, up, k = gather(trajs, items, net.dev)
            net.features(un, um, k, up)
            loss = net.train_step(net.B, lr=lr)
            tot += float(loss.item())
            nb_tot += 1
        losses.append(tot / max(nb_tot, 1))
        if log:
            log("epoch %d loss %.4e" % (ep, losses[-1]))
    return losses


def evaluate(plan, net: WarmStartNet, trajs, tol=1e-10):
    """Replays held-out steps: PSD from the extrapolated guess and from the
    learned guess, identical inputs, same tolerance.  Returns per-step
    iteration counts and wall times (learned time includes inference and the
    forward transform of the guess)."""
    dev = plan.device
    rows = []
    for S, ks in trajs:
        for n in range(1, S.shape[0] - 1):
            k1, k0 = float(ks[n + 1]), float(ks[n])
            uhn = plan.forward(S[n].contiguous())
            uhm = plan.forward(S[n - 1].contiguous())
            # inputs of both solves are prepared outside the timed regions
            k = torch.tensor([[k1, k0]], dtype=torch.float64, device=dev)
            s_n, s_m = S[n:n + 1].contiguous(), S[n - 1:n].contiguous()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sol_plain, st_plain = plan.step_psd(uhn, uhm, k1, k0, tol=tol, max_iter=4000,
                                                raise_noconv=False)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            g = net.guess(s_n, s_m, k)
            gh = plan.forward(g[0].contiguous())
            sol_learn, st_learn = plan.step_psd(uhn, uhm, k1, k0, guess=gh, tol=tol,
                                                max_iter=4000, raise_noconv=False)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            diff = float(torch.linalg.norm(sol_learn - sol_plain) / torch.linalg.norm(sol_plain))
            rows.append((st_plain["iters"], st_learn["iters"], t1 - t0, t2 - t1, diff))
    a = np.array(rows, dtype=float)
    # 4 FFT calls per PSD iteration; the learned step also transforms its guess
    return {"steps": len(rows), "iters_plain": float(a[:, 0].mean()),
            "iters_learned": float(a[:, 1].mean()),
            "fft_calls_per_step_plain": 4.0 * float(a[:, 0].mean()),
            "fft_calls_per_step_learned": 4.0 * float(a[:, 1].mean()) + 1.0,
            "ms_per_step_plain": 1e3 * float(a[:, 2].mean()),
            "ms_per_step_learned": 1e3 * float(a[:, 3].mean()),
            "max_rel_diff_solutions": float(a[:, 4].max()),
            "per_step": rows}


def run_experiment(train_seeds, test_seeds, nsteps=60, epochs=20, batch=16, lr=1e-3,
                   tol=1e-10, log=None, device="cuda:0", t_burn=0.0):
    kw = c5_model()
    plan = fch.Plan(**kw, device=device)
    t0 = time.perf_counter()
    tr, te = [], []
    for dst, seeds in ((tr, train_seeds), (te, test_seeds)):
        for s in seeds:
            dst.append(psd_trajectory(plan, c5_initial(s), nsteps, tol=tol, t_burn=t_burn))
            if log:
                log("trajectory seed %d: %d steps to t = %.3f" % (s, dst[-1][0].shape[0] - 1,
                                                                  float(dst[-1][1].sum())))
    t_gen = time.perf_counter() - t0
    if log:
        log("generated %d + %d trajectories in %.1fs" % (len(tr), len(te), t_gen))
    net = WarmStartNet(kw["N"], kw["N"], batch, seed=0, device=device)
    t0 = time.perf_counter()
    losses = train(net, tr, epochs=epochs, lr=lr, log=log)
    t_train = time.perf_counter() - t0
    ev = evaluate(plan, net, te, tol=tol)
    ev.update({"train_pairs": len(make_pairs(tr)), "epochs": epochs, "loss_first": losses[0],
               "loss_last": losses[-1], "gen_s": round(t_gen, 2), "train_s": round(t_train, 2)})
    return ev, net, plan


# parameters trained at the full scale of the warm-start workload (40 seeds x
# 500 accepted steps, 10 epochs), written by `python -m
# paper_2006_04784_amd.learned --train-full <path>`
WEIGHTS_C5 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                          "warm_start_c5_full.npz")


def evaluate_pretrained(weights, test_seeds, nsteps=500, tol=1e-10, log=None, device="cuda:0"):
    """Held-out comparison with stored parameters: generates the test
    trajectories (full length), then replays every step plainly and from the
    learned guess (evaluate)."""
    kw = c5_model()
    plan = fch.Plan(**kw, device=device)
    net = WarmStartNet(kw["N"], kw["N"], 1, seed=0, device=device)
    net.load_params(weights)
    t0 = time.perf_counter()
    te = []
    for s in test_seeds:
        te.append(psd_trajectory(plan, c5_initial(s), nsteps, tol=tol))
        if log:
            log("trajectory seed %d: %d steps to t = %.3f" % (s, te[-1][0].shape[0] - 1,
                                                              float(te[-1][1].sum())))
    t_gen = time.perf_counter() - t0
    ev = evaluate(plan, net, te, tol=tol)
    ev.update({"gen_s": round(t_gen, 2), "weights": os.path.basename(weights)})
    return ev


def _main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="learned PSD warm start at 256^2")
    ap.add_argument("--train-full", metavar="PATH",
                    help="generate 40 x 500-step training trajectories, train 10 epochs and "
                         "write the parameters to PATH")
    ap.add_argument("--seeds", type=int, default=40)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--epochs", type=int, default=10)
    args = ap.parse_args(argv)
    if args.train_full:
        def log(m):
            print(m, flush=True)
        ev, net, _ = run_experiment(range(args.seeds), [900, 901], nsteps=args.steps,
                                    epochs=args.epochs, log=log)
        net.save_params(args.train_full)
        ev.pop("per_step")
        print({k: v for k, v in ev.items()}, flush=True)


if __name__ == "__main__":
    _main()
