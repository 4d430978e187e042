"""GPU adaptive runs replayed by the oracle at the workloads' own shapes.

- Adaptive BDF2-PSD (Sec. 3.2 controller with the Sec. 3.3 solver) on a 256^2
  field of the 2048^2 workload's kind (perturbed loops plus a Gaussian random
  field): every attempt, rejected ones included, is replayed on the oracle
  with the GPU's trial step and PSD iteration count; the AM3 estimate, the
  accept decision (outside the tie zone |e - sigma|/sigma < 1e-9) and the
  next step agree, and so does the state.  The library's own adaptive driver
  (fch_run) takes the same attempts.
- The 2048^2 workload itself (forty loops plus the random field, sigma_tol
  1e-6, i_tol 1e-10, k_max 0.05, lambda from Table SearchSize): the startup
  step and the first accepted steps, replayed the same way.
- A 1024^2 member of the mixed-size ensemble: its device-chosen steps
  replayed on the oracle's IMEX stepper and its AM3 estimate.
"""
import os
import sys

import numpy as np
import pytest
import torch

from paper_2006_04784_amd import inputs

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_04784_amd import fch
    fch.lib()
    return fch


@pytest.fixture(scope="module")
def orc_mt(orc):
    orc.set_threads(min(16, os.cpu_count() or 1))
    yield orc
    orc.set_threads(1)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(uh_np):
    return torch.from_numpy(np.ascontiguousarray(uh_np.T)).to("cuda")


def host(uh_t):
    return uh_t.cpu().numpy().T


def sav_free_kw(kw):
    L = kw["L"]
    return dict(kw, p=1, q=0.0, zeta=1.1, D0=L * L * 1.05)


def gpu_adaptive_psd(F, plan, u0_dev, opts, k_first, tol, n_accept):
    """Sec. 3.2 Steps 0-4 driven from the host over the library's calls:
    startup PSD step of k_first (first order), then attempts until n_accept
    steps are accepted.  Returns the attempts (k, iterations, e, accept,
    k_next), the startup iterations and the final state."""
    Fm = plan.rhs(u0_dev)
    cur, st = plan.step_psd(u0_dev, u0_dev, k_first, -1.0, tol=tol)
    it0 = st["iters"]
    prev = u0_dev
    Fn = plan.rhs(cur)
    kn, kt, t = k_first, k_first, k_first
    attempts = []
    acc_n = 1
    while acc_n < n_accept:
        trial, st = plan.step_psd(cur, prev, kt, kn, tol=tol)
        Ft, acc, knext, e = plan.adapt_dt(trial, cur, Fn, Fm, kt, kn, opts)
        attempts.append((kt, st["iters"], e, acc, knext))
        if acc:
            prev, cur = cur, trial
            Fm, Fn = Fn, Ft
            t += kt
            kn = kt
            acc_n += 1
        kt = knext
    return attempts, it0, cur, prev, t


def oracle_replay_psd(orc, m, uh0, k_first, it0, attempts, sigma, k_min, k_max, tol):
    """Replays every GPU attempt on the oracle with the GPU's step and PSD
    iteration count; returns the oracle's final state and the largest
    relative differences of e and k_next."""
    cur, _, _, _ = orc.psd_step(m, uh0, None, k_first, -1.0, fixed_iters=it0)
    prev = uh0
    Fm, Fn = orc.F(m, prev), orc.F(m, cur)
    kn = k_first
    de = dk = 0.0
    for (kt, it, e_gpu, acc_gpu, knext_gpu) in attempts:
        trial, _, _, _ = orc.psd_step(m, cur, prev, kt, kn, fixed_iters=it)
        Ft = orc.F(m, trial)
        e = orc.am3_error(m, trial, cur, Ft, Fn, Fm, kt, kn)
        acc, knext = orc.adapt_decide(e, kt, sigma, k_min, k_max)
        de = max(de, abs(e_gpu / e - 1.0))
        dk = max(dk, abs(knext_gpu / knext - 1.0))
        if abs(e - sigma) / sigma > 1e-9:
            assert acc == acc_gpu, (kt, e, e_gpu)
        if acc_gpu:
            prev, cur = cur, trial
            Fm, Fn = Fn, Ft
            kn = kt
    return cur, de, dk


def test_adaptive_psd_replayed_by_oracle(F, orc_mt):
    orc = orc_mt
    kw, u0 = inputs.psd_mix(256, seed=4)
    kw = sav_free_kw(kw)
    plan = F.Plan(**kw)
    m = orc.Model(**kw)
    sigma, k_min, k_max, tol, k_first = 1e-5, 1e-9, 0.05, 1e-10, 1e-9
    opts = F.AdaptOpts(sigma_tol=sigma, k_min=k_min, k_max=k_max)
    uh0 = orc.r2c(u0)
    log("adaptive PSD 256^2 (loops + random field): GPU attempts")
    attempts, it0, cur, prev, t = gpu_adaptive_psd(F, plan, dev(uh0), opts, k_first, tol, 40)
    n_rej = sum(1 for a in attempts if not a[3])
    iters = it0 + sum(a[1] for a in attempts)
    log("  %d attempts (%d rejected), %d PSD iterations, t = %.4g, last k %.3g"
        % (len(attempts), n_rej, iters, t, attempts[-1][0]))
    log("oracle replay")
    o_cur, de, dk = oracle_replay_psd(orc, m, uh0, k_first, it0, attempts, sigma, k_min, k_max,
                                      tol)
    e_state = rel(host(cur), o_cur)
    log("  state rel %.3e, max |e_gpu/e_oracle - 1| %.3e, max |k_next ratio - 1| %.3e"
        % (e_state, de, dk))
    # measured: state 5.7e-16, e 6.0e-11, k_next 7.5e-13 (39 attempts)
    assert e_state < 1e-8
    assert de < 1e-8 and dk < 1e-8
    assert attempts[-1][0] > 100 * k_first
    # the library's adaptive driver takes the same attempts to the same state
    a = dev(uh0)
    b = torch.zeros_like(a)
    info = plan.run(a, b, scheme="psd", adaptive=True, startup=True, t_end=t, k_first=k_first,
                    adapt=opts, nsteps=40, psd_tol=tol)
    assert info["accepted"] == 40 and info["rejected"] == n_rej
    assert info["psd_iters"] == iters
    assert rel(host(a), host(cur)) < 1e-12 and rel(host(b), host(prev)) < 1e-12


def test_c3_2048_first_steps_replayed_by_oracle(F, orc_mt):
    orc = orc_mt
    log("c3 2048^2 input (40 loops + random field)")
    kw, u0 = inputs.workload("c3")
    kw = dict(kw, p=1, q=0.0)
    z, d0 = F.sav_constants(F.fch_params(kw["N"], kw["L"], kw["eps"], kw["eta1"], kw["eta2"], 1,
                                         0.0, 0.3, -1.0, 1.0, 2.0, 1.0, 0.0, 0.0))
    kw = dict(kw, zeta=z, D0=d0)
    plan = F.Plan(**kw)
    m = orc.Model(**kw)
    sigma, k_min, k_max, tol, k_first = 1e-6, 1e-9, 0.05, 1e-10, 1e-9
    opts = F.AdaptOpts(sigma_tol=sigma, k_min=k_min, k_max=k_max)
    uh0 = orc.r2c(u0)
    log("  GPU: startup and 2 accepted steps")
    attempts, it0, cur, prev, t = gpu_adaptive_psd(F, plan, dev(uh0), opts, k_first, tol, 3)
    log("  attempts %s, startup iterations %d" % ([(a[0], a[1], a[3]) for a in attempts], it0))
    log("  oracle replay")
    o_cur, de, dk = oracle_replay_psd(orc, m, uh0, k_first, it0, attempts, sigma, k_min, k_max,
                                      tol)
    e_state = rel(host(cur), o_cur)
    log("  state rel %.3e, max |e ratio - 1| %.3e, max |k_next ratio - 1| %.3e"
        % (e_state, de, dk))
    # measured: state 5.3e-17, e 3.7e-12, k_next 0
    assert e_state < 1e-8
    assert de < 1e-8 and dk < 1e-8
    a = dev(uh0)
    b = torch.zeros_like(a)
    info = plan.run(a, b, scheme="psd", adaptive=True, startup=True, t_end=t, k_first=k_first,
                    adapt=opts, nsteps=3, psd_tol=tol)
    assert info["accepted"] == 3
    assert rel(host(a), host(cur)) < 1e-12


def test_c4_1024_member_replayed_by_oracle(F, orc_mt):
    orc = orc_mt
    mem_all = inputs.c4_members()
    idx = [i for i, mm in enumerate(mem_all) if mm["N"] == 1024][0]
    small = [i for i, mm in enumerate(mem_all) if mm["N"] == 128][0]
    sel = [idx, small]
    mem = [sav_free_kw(mem_all[i]) for i in sel]
    log("c4 members %s (N = %s): 6 accepted steps" % (sel, [mm["N"] for mm in mem]))
    ens = F.Ensemble(mem, adapt=F.AdaptOpts(sigma_tol=1e-5), t_end=1e9, max_steps=6)
    for j, i in enumerate(sel):
        ens.load(j, torch.from_numpy(inputs.c4_initial(mem_all[i], i)).cuda())
    ens.run(max_attempts=200, sync_every=10, use_graph=True)
    for j, i in enumerate(sel):
        uh, klog, mi = ens.member(j)
        assert mi["accepted"] == 6 and mi["done"]
        m = orc.Model(**mem[j])
        u0 = orc.r2c(inputs.c4_initial(mem_all[i], i))
        prev, cur = u0, orc.imex_step(m, u0, None, klog[0], -1.0)
        Fm, Fn = orc.F(m, prev), orc.F(m, cur)
        for s in range(1, len(klog)):
            nxt = orc.imex_step(m, cur, prev, klog[s], klog[s - 1])
            Ft = orc.F(m, nxt)
            e = orc.am3_error(m, nxt, cur, Ft, Fn, Fm, klog[s], klog[s - 1])
            acc, _ = orc.adapt_decide(e, klog[s], 1e-5, 1e-9, np.inf)
            assert acc or abs(e - 1e-5) / 1e-5 < 1e-9
            prev, cur, Fm, Fn = cur, nxt, Fn, Ft
        e_state = rel(host(uh), cur)
        log("  member %d (N=%d): steps %s, state rel %.3e"
            % (i, mem[j]["N"], ["%.3g" % k for k in klog], e_state))
        assert e_state < 1e-8


def dyadic_next(accept, e_next, kt, jt, tu, kb, kmin, kmax, clamped, jmin=-24, jmax=38):
    """The nested factor-of-two rule: (next ladder index, accepted time in units
    of kb 2^jmin) from the step law's proposal e_next after an attempt of kt."""
    lad = lambda j: kb * 2.0 ** j
    jn = jt
    if accept and not clamped:
        tu += 1 << (jt - jmin)
        if e_next >= 2 * kt and jt < jmax and tu % (1 << (jt + 1 - jmin)) == 0:
            jn = jt + 1
        elif e_next < kt:
            while jn > jmin and lad(jn) > e_next:
                jn -= 1
    elif not accept:
        jn = jt - 1
        while jn > jmin and lad(jn) > e_next:
            jn -= 1
    while jn > jmin and lad(jn) > kmax:
        jn -= 1
    while jn < jt and lad(jn) < kmin:
        jn += 1
    return jn, tu


def test_nested_dyadic_sav_follows_the_oracle_controller(F, orc_mt):
    """Adaptive SAV with nested factor-of-two steps (fch_run dyadic) on a 128^2
    circle: the oracle's SAV steps and AM3 estimate driven by the same ladder
    rule accept the same number of steps, reach the same time and the same
    state and r; the ladder costs more FFT calls than the plain step law."""
    orc = orc_mt
    N, L, T = 128, 2 * np.pi, 0.02
    kw = dict(N=N, L=L, eps=0.1, eta1=1.45, eta2=2.0, p=1, q=0.0, zeta=1.1, D0=L * L * 1.05)
    plan = F.Plan(**kw)
    m = orc.Model(**kw)
    uh0 = orc.r2c(inputs.circle_bilayer(N, L, 0.1, seed=7))
    sigma, kmin, kb = 1e-5, 1e-9, 1e-9
    opts = F.AdaptOpts(sigma_tol=sigma, k_min=kmin)
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    plan.reset_stats()
    info = plan.run(a, b, scheme="sav", adaptive=True, startup=True, t_end=T, k_first=kb,
                    adapt=opts, nsteps=10 ** 7, dyadic=True)
    calls_dyadic = plan.stats()["fft_calls"]
    a2, b2 = dev(uh0), torch.zeros_like(dev(uh0))
    plan.reset_stats()
    info2 = plan.run(a2, b2, scheme="sav", adaptive=True, startup=True, t_end=T, k_first=kb,
                     adapt=opts, nsteps=10 ** 7)
    calls_plain = plan.stats()["fft_calls"]
    log("nested dyadic SAV: %d accepted, %d rejected, %d FFT calls; step law: %d accepted, "
        "%d FFT calls (ratio %.2f)" % (info["accepted"], info["rejected"], calls_dyadic,
                                       info2["accepted"], calls_plain, calls_dyadic / calls_plain))
    # the oracle with the same rule
    r0 = float(np.sqrt(orc.E1(m, uh0) + m.D0))
    prev = uh0
    cur, r_cur = orc.sav_step(m, prev, None, r0, r0, kb, -1.0)
    r_prev = r0
    Fm, Fn = orc.F(m, prev), orc.F(m, cur)
    t, kn, jt, tu = kb, kb, 0, 1 << 24
    acc_n, rej_n = 1, 0
    while t < T * (1 - 1e-14):
        kt = kb * 2.0 ** jt
        clamped = kt > T - t
        if clamped:
            kt = T - t
        trial, r_trial = orc.sav_step(m, cur, prev, r_cur, r_prev, kt, kn)
        Ft = orc.F(m, trial)
        e = orc.am3_error(m, trial, cur, Ft, Fn, Fm, kt, kn)
        ok, knext = orc.adapt_decide(e, kt, sigma, kmin, np.inf)
        assert abs(e - sigma) / sigma > 1e-9   # outside the tie zone
        jt, tu = dyadic_next(ok, knext, kt, jt, tu, kb, kmin, np.inf, clamped)
        if ok:
            prev, cur, Fm, Fn = cur, trial, Fn, Ft
            r_prev, r_cur = r_cur, r_trial
            t, kn = t + kt, kt
            acc_n += 1
        else:
            rej_n += 1
    e_state = rel(host(a), cur)
    log("  oracle: %d accepted, %d rejected; state rel %.3e, r rel %.3e"
        % (acc_n, rej_n, e_state, abs(info["rs"][0] - r_cur) / abs(r_cur)))
    assert info["accepted"] == acc_n and info["rejected"] == rej_n
    assert abs(info["t"] - t) < 1e-12
    assert e_state < 1e-8
    assert abs(info["rs"][0] - r_cur) < 1e-10 * abs(r_cur)
    assert calls_dyadic > calls_plain
