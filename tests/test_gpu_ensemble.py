"""GPU tests of the batched ensemble (device-side adaptive step control in
captured HIP graphs): each member against an independent single run and the
oracle, graph replay against eager launches, and mixed grid sizes."""
import sys

import numpy as np
import pytest
import torch

from paper_2006_04784_amd import inputs

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_04784_amd import fch
    fch.lib()
    return fch


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def members_small():
    out = []
    for i, (N, e1, e2) in enumerate([(64, 1.45, 2.0), (128, 1.3, 1.7), (64, 1.55, 2.3),
                                     (128, 1.2, 2.5), (32, 1.5, 1.9)]):
        L = N * 4 * np.pi / 256 if N >= 64 else 2 * np.pi
        out.append(dict(N=N, L=L, eps=0.1, eta1=e1, eta2=e2, zeta=1.1, D0=L * L * 1.05))
    return out


def initial(m, seed):
    return inputs.circle_bilayer(m["N"], m["L"], m["eps"], seed=seed)


def build(F, mem, use_max=40, t_end=10.0):
    ens = F.Ensemble(mem, adapt=F.AdaptOpts(sigma_tol=1e-5), t_end=t_end, max_steps=use_max)
    for i, m in enumerate(mem):
        ens.load(i, torch.from_numpy(initial(m, seed=10 + i)).cuda())
    return ens


def test_ensemble_members_match_single_runs(F):
    log("ensemble vs single runs")
    mem = members_small()
    ens = build(F, mem)
    info = ens.run(max_attempts=1000, sync_every=7, use_graph=True)
    assert info["active"] == 0
    for i, m in enumerate(mem):
        uh, klog, mi = ens.member(i)
        assert mi["done"] and mi["accepted"] == 40 and not mi["nonfinite"]
        plan = F.Plan(**m)
        a = plan.forward(torch.from_numpy(initial(m, seed=10 + i)).cuda())
        b = torch.empty_like(a)
        ri = plan.run(a, b, scheme="imex", adaptive=True, startup=True, t_end=10.0,
                      adapt=F.AdaptOpts(sigma_tol=1e-5), nsteps=40)
        assert ri["accepted"] == mi["accepted"]
        assert rel(uh.cpu().numpy(), a.cpu().numpy()) < 1e-12
        assert abs(ri["t"] - mi["t"]) < 1e-12 * ri["t"]


def test_ensemble_member_replayed_by_oracle(F, orc):
    log("ensemble member oracle replay")
    mem = members_small()[:2]
    ens = build(F, mem, use_max=30)
    ens.run(max_attempts=500, sync_every=5, use_graph=True)
    for i, m in enumerate(mem):
        uh, klog, mi = ens.member(i)
        om = orc.Model(**m)
        u0 = orc.r2c(initial(m, seed=10 + i))
        prev, cur = u0, orc.imex_step(om, u0, None, klog[0], -1.0)
        for j in range(1, len(klog)):
            prev, cur = cur, orc.imex_step(om, cur, prev, klog[j], klog[j - 1])
        assert len(klog) == 30 and klog[-1] > 100 * klog[0]
        assert rel(uh.cpu().numpy().T, cur) < 1e-8


def test_graph_replay_equals_eager(F):
    log("ensemble graph vs eager")
    mem = members_small()
    e1 = build(F, mem, use_max=25)
    e1.run(max_attempts=1000, sync_every=1, use_graph=False)
    e2 = build(F, mem, use_max=25)
    # several replays, each followed by the host's own read-back and sync
    for _ in range(200):
        info = e2.run(max_attempts=1, sync_every=1, use_graph=True)
        torch.cuda.synchronize()
        if info["active"] == 0:
            break
    for i in range(len(mem)):
        u1, k1, m1 = e1.member(i)
        u2, k2, m2 = e2.member(i)
        assert m1["accepted"] == m2["accepted"] and m1["rejected"] == m2["rejected"]
        assert np.array_equal(k1, k2)
        assert torch.equal(u1, u2)


def test_mixed_sizes_autotuned(F):
    log("ensemble mixed sizes autotuned")
    rng = np.random.default_rng(7)
    mem = []
    for N in (256, 128, 512, 256):
        L = N * 4 * np.pi / 256
        mem.append(dict(N=N, L=L, eps=0.1, eta1=rng.uniform(1.2, 1.6),
                        eta2=rng.uniform(1.5, 2.5)))
    ens = build(F, mem, use_max=20)
    ens.autotune(reps=2)
    info = ens.run(max_attempts=1000, sync_every=10, use_graph=True)
    assert info["active"] == 0 and info["accepted"] == 20 * len(mem)
    for i, m in enumerate(mem):
        uh, klog, mi = ens.member(i)
        assert torch.isfinite(uh).all() and mi["accepted"] == 20


def test_ensemble_step_queues_without_waiting(F):
    """fch_ensemble_step: attempts queued in chunks (graph and eager) reach
    the same member states, bit for bit, as one fch_ensemble_run."""
    log("ensemble step chunks")
    mem = members_small()
    ref = build(F, mem)
    ref.run(max_attempts=1000, sync_every=50, use_graph=True)
    for use_graph in (True, False):
        ens = build(F, mem)
        for _ in range(40):   # more attempts than any member needs: finished ones idle
            ens.step(attempts=5, use_graph=use_graph)
        info = ens.run(max_attempts=1, sync_every=1, use_graph=use_graph)
        for i in range(len(mem)):
            a, ka, ma = ens.member(i)
            b, kb, mb = ref.member(i)
            assert ma["done"] and ma["accepted"] == mb["accepted"], (use_graph, i)
            assert torch.equal(a, b) and np.array_equal(ka, kb), (use_graph, i)


def test_running_max_of_u(F):
    """Each member's umax is the running maximum of u over its accepted states
    (the trial evaluation's row pass records the largest u per workgroup and
    the controller folds it in on acceptance), checked one attempt at a time
    against the inverse transform of the member's current state."""
    log("ensemble running max of u")
    mem = members_small()[:3]
    ens = build(F, mem, use_max=30)
    plans = {m["N"]: F.Plan(**m) for m in mem}
    run_max = [-np.inf] * len(mem)
    last = [1] * len(mem)
    for _ in range(40):
        ens.step(1, use_graph=False)
        for i, m in enumerate(mem):
            uh, _, mi = ens.member(i, klog=False)
            if mi["accepted"] > last[i]:
                run_max[i] = max(run_max[i], float(plans[m["N"]].inverse(uh).max()))
                last[i] = mi["accepted"]
            if run_max[i] == -np.inf:
                assert mi["umax"] == -np.inf
            else:
                assert abs(mi["umax"] - run_max[i]) <= 1e-12 * abs(run_max[i]), (i, mi, run_max[i])
    assert all(np.isfinite(run_max))


def test_defect_onset_dichotomy(F):
    """The critical benchmark (Table t:Benchmark) with the paper's initial data
    below and above the onset of defects (Sec. 5.1): after the initial
    relaxation the maximum of u sits at the bilayer's peak, which the paper
    puts at u = 0.3566, or near a defect's, about 0.74."""
    log("defect onset dichotomy, critical benchmark 256^2")
    from paper_2006_04784_amd import sweeps
    res = sweeps.critical_d_sweep([0.745, 0.775], sigma_tol=1e-5, t_end=60.0, t0=45.0)
    lo, hi = res["umax"]
    assert abs(lo - 0.3566) < 0.005, res
    assert 0.70 < hi < 0.80, res
    assert res["d_critical"] == 0.775 and res["d_max_without_defect"] == 0.745


def build_scheme(F, mem, scheme, use_max=30, t_end=10.0):
    ens = F.Ensemble(mem, adapt=F.AdaptOpts(sigma_tol=1e-5), t_end=t_end, max_steps=use_max,
                     scheme=scheme)
    for i, m in enumerate(mem):
        ens.load(i, torch.from_numpy(initial(m, seed=10 + i)).cuda())
    return ens


@pytest.mark.parametrize("scheme", ["sav", "etd"])
def test_ensemble_schemes_match_single_runs(F, scheme):
    """SAV and ETDRK2 members of an ensemble reach the states, times and step
    counts of independent single-plan adaptive runs of the same scheme (both
    take the first-order startup step k_min; ETDRK2's single run evaluates its
    first stage with the cached F(u^0), which rounds differently)."""
    log("ensemble %s vs single runs" % scheme)
    mem = members_small()
    ens = build_scheme(F, mem, scheme)
    info = ens.run(max_attempts=1000, sync_every=7, use_graph=True)
    assert info["active"] == 0
    tol = 1e-12 if scheme == "sav" else 1e-10
    for i, m in enumerate(mem):
        uh, klog, mi = ens.member(i)
        assert mi["done"] and mi["accepted"] == 30 and not mi["nonfinite"] and not mi["invalid"]
        plan = F.Plan(**m)
        a = plan.forward(torch.from_numpy(initial(m, seed=10 + i)).cuda())
        b = torch.empty_like(a)
        ri = plan.run(a, b, scheme=scheme, adaptive=True, startup=True, t_end=10.0,
                      adapt=F.AdaptOpts(sigma_tol=1e-5), nsteps=30)
        assert ri["accepted"] == mi["accepted"], (i, ri, mi)
        assert rel(uh.cpu().numpy(), a.cpu().numpy()) < tol, i
        assert abs(ri["t"] - mi["t"]) < tol * ri["t"]
        if scheme == "sav":
            assert abs(ri["rs"][0] - mi["r_n"]) < tol * abs(mi["r_n"])
            assert abs(ri["rs"][1] - mi["r_nm1"]) < tol * abs(mi["r_nm1"])
        else:
            assert mi["r_n"] == 0.0 and mi["r_nm1"] == 0.0


@pytest.mark.parametrize("scheme", ["sav", "etd"])
def test_ensemble_scheme_member_replayed_by_oracle(F, orc, scheme):
    """The accepted step sizes of an ensemble member, replayed by the oracle's
    steppers from the same initial data, reproduce the member's state (and,
    for SAV, its r)."""
    log("ensemble %s member oracle replay" % scheme)
    mem = members_small()[:2]
    ens = build_scheme(F, mem, scheme, use_max=25)
    ens.run(max_attempts=500, sync_every=5, use_graph=True)
    for i, m in enumerate(mem):
        uh, klog, mi = ens.member(i)
        om = orc.Model(**m)
        u0 = orc.r2c(initial(m, seed=10 + i))
        assert len(klog) == 25 and klog[-1] > 10 * klog[0]
        if scheme == "sav":
            r0 = float(np.sqrt(orc.E1(om, u0) + om.D0))
            cur, r1 = orc.sav_step(om, u0, None, r0, r0, klog[0], -1.0)
            prev, rp = u0, r0
            rc = r1
            for j in range(1, len(klog)):
                nxt, rn = orc.sav_step(om, cur, prev, rc, rp, klog[j], klog[j - 1])
                prev, rp, cur, rc = cur, rc, nxt, rn
            assert abs(rc - mi["r_n"]) < 1e-8 * abs(rc)
            assert abs(rp - mi["r_nm1"]) < 1e-8 * abs(rp)
        else:
            cur = u0
            for k in klog:
                cur = orc.etd_step(om, cur, k)
        assert rel(uh.cpu().numpy().T, cur) < 1e-8, i


@pytest.mark.parametrize("scheme", ["sav", "etd"])
def test_ensemble_scheme_mixed_sizes_autotuned(F, scheme):
    """Mixed grid sizes after the autotuner picked each class's variants (the
    SAV row pass's partial count follows the chosen variant): every member
    still matches an independent single run."""
    log("ensemble %s mixed sizes autotuned" % scheme)
    rng = np.random.default_rng(11)
    mem = []
    for N in (256, 128, 512):
        L = N * 4 * np.pi / 256
        mem.append(dict(N=N, L=L, eps=0.1, eta1=rng.uniform(1.2, 1.6),
                        eta2=rng.uniform(1.5, 2.5)))
    ens = build_scheme(F, mem, scheme, use_max=12)
    ens.autotune(reps=2)
    info = ens.run(max_attempts=1000, sync_every=10, use_graph=True)
    assert info["active"] == 0 and info["accepted"] == 12 * len(mem)
    tol = 1e-12 if scheme == "sav" else 1e-10
    for i, m in enumerate(mem):
        uh, klog, mi = ens.member(i)
        plan = F.Plan(**m)
        a = plan.forward(torch.from_numpy(initial(m, seed=10 + i)).cuda())
        b = torch.empty_like(a)
        ri = plan.run(a, b, scheme=scheme, adaptive=True, startup=True, t_end=10.0,
                      adapt=F.AdaptOpts(sigma_tol=1e-5), nsteps=12)
        assert ri["accepted"] == mi["accepted"] == 12
        assert rel(uh.cpu().numpy(), a.cpu().numpy()) < tol, i


@pytest.mark.parametrize("scheme", ["imex", "sav"])
def test_autotune_restores_members(F, scheme):
    """The batched autotuner runs whole attempts of each class's members for
    every variant pair, then restores them: states, step logs and counters
    are bit for bit those before tuning, and a run after tuning matches an
    untuned one to rounding with the same step counts."""
    log("ensemble %s autotune restores members" % scheme)
    mem = members_small()
    ens = build_scheme(F, mem, scheme, use_max=20)
    before = [ens.member(i) for i in range(len(mem))]
    ens.autotune(reps=2)
    for i in range(len(mem)):
        u, k, mi = ens.member(i)
        u0, k0, m0 = before[i]
        assert torch.equal(u, u0) and np.array_equal(k, k0), i
        assert mi == m0, (i, mi, m0)
    ens.run(max_attempts=1000, sync_every=10, use_graph=True)
    ref = build_scheme(F, mem, scheme, use_max=20)
    ref.run(max_attempts=1000, sync_every=10, use_graph=True)
    for i in range(len(mem)):
        u, k, mi = ens.member(i)
        r, kr, mr = ref.member(i)
        assert mi["accepted"] == mr["accepted"] == 20 and mi["rejected"] == mr["rejected"], i
        assert rel(u.cpu().numpy(), r.cpu().numpy()) < 1e-10, i
        assert np.allclose(k, kr, rtol=1e-9, atol=0), i


@pytest.mark.parametrize("N", [256, 1024])
def test_device_control_every_variant(F, N):
    """The batched stage kernels under every compiled (row, column) variant
    pair: a device-controlled adaptive run (a one-member ensemble) of each
    scheme gives the default variant's state and step counts to rounding."""
    log("device control, every variant N=%d" % N)
    rows, cols = F.config_list(N)
    L = N * 4 * np.pi / 256
    plan = F.Plan(N=N, L=L, eps=0.1, eta1=1.4, eta2=2.0)
    u0 = torch.from_numpy(inputs.circle_bilayer(N, L, 0.1, seed=10)).cuda()

    def go(scheme, cfg):
        plan.set_config(cfg)
        a = plan.forward(u0)
        b = torch.empty_like(a)
        ri = plan.run(a, b, scheme=scheme, adaptive=True, startup=True, t_end=10.0,
                      adapt=F.AdaptOpts(sigma_tol=1e-5), nsteps=6)
        return a.cpu().numpy(), ri

    for scheme in ("imex", "sav", "etd"):
        ref, rr = go(scheme, None)
        for r in rows:
            for c in cols:
                x, ri = go(scheme, r + c)
                assert ri["accepted"] == rr["accepted"] and ri["rejected"] == rr["rejected"]
                assert rel(x, ref) < 1e-12, (scheme, r, c)


def test_ensemble_rejects_bad_scheme_options(F):
    """PSD is not batched, and ETDRK2's stabilizers must be finite and >= 0:
    fch_ensemble_create returns FCH_E_INVALID and creates nothing."""
    import ctypes as C
    log("ensemble bad scheme options")
    m = members_small()[0]
    prm = F.fch_params(m["N"], m["L"], m["eps"], m["eta1"], m["eta2"], 1, 0.0, 0.3, -1.0, 1.0,
                       2.0, 1.0, m["zeta"], m["D0"])
    arr = (F.fch_params * 1)(prm)
    for scheme, k0, k2 in ((F.FCH_PSD, 0.01, 15.0), (7, 0.01, 15.0), (F.FCH_ETD, -1.0, 15.0),
                           (F.FCH_ETD, 0.01, float("nan")), (F.FCH_ETD, float("inf"), 15.0)):
        o = F.fch_ensemble_opts(F.AdaptOpts().c(), 1.0, 10, 0.0, 0.0, scheme,
                                F.fch_etd_opts(k0, k2))
        h = C.c_void_p()
        assert F.lib().fch_ensemble_create(arr, 1, C.byref(o), C.byref(h)) == F.FCH_E_INVALID
        assert not h.value
    with pytest.raises(ValueError):
        F.Ensemble([m], scheme="psd")


def test_ensemble_extreme_sizes_and_degenerate_runs(F):
    """The smallest and the largest grids in one ensemble (16^2 and 4096^2,
    their own classes), next to degenerate members: one whose t_end is reached
    by the startup step alone and one whose cap (max_steps = 2) allows one
    adaptive step.  Each matches an independent single run."""
    log("ensemble 16^2 + 4096^2 + degenerate members")
    mem = [dict(N=16, L=2 * np.pi, eps=0.3, eta1=1.45, eta2=2.0),
           dict(N=4096, L=16 * np.pi, eps=0.1, eta1=1.4, eta2=2.1)]
    for kw in (dict(t_end=1e-9, max_steps=5), dict(t_end=10.0, max_steps=2)):
        ens = F.Ensemble(mem, adapt=F.AdaptOpts(sigma_tol=1e-5), k_first=1e-6, **kw)
        u0s = [torch.from_numpy(inputs.circle_bilayer(m["N"], m["L"], m["eps"], seed=4 + i)).cuda()
               for i, m in enumerate(mem)]
        for i, u in enumerate(u0s):
            ens.load(i, u)
        info = ens.run(max_attempts=50, sync_every=5, use_graph=True)
        assert info["active"] == 0, kw
        for i, m in enumerate(mem):
            uh, klog, mi = ens.member(i)
            plan = F.Plan(**m)
            a = plan.forward(u0s[i])
            b = torch.empty_like(a)
            ri = plan.run(a, b, scheme="imex", adaptive=True, startup=True, t_end=kw["t_end"],
                          k_first=1e-6, adapt=F.AdaptOpts(sigma_tol=1e-5),
                          nsteps=kw["max_steps"])
            assert mi["done"] and mi["accepted"] == ri["accepted"], (kw, i, mi, ri)
            if kw["t_end"] < 1e-6:
                assert mi["accepted"] == 1 and mi["t"] == kw["t_end"]   # clamped startup
            else:
                assert mi["accepted"] == 2
            assert rel(uh.cpu().numpy(), a.cpu().numpy()) < 1e-12, (kw, i)
        ens.close()


@pytest.mark.parametrize("scheme", ["sav", "etd"])
def test_scheme_graph_replay_and_queued_steps_equal_eager(F, scheme):
    """SAV and ETDRK2 ensembles: graph replays (run and queued fch_ensemble_step
    chunks, with the host's own syncs between them) reach the eager launches'
    states, step logs, counters and SAV scalars bit for bit."""
    log("ensemble %s graph / queued / eager" % scheme)
    mem = members_small()
    ref = build_scheme(F, mem, scheme, use_max=25)
    ref.run(max_attempts=1000, sync_every=1, use_graph=False)
    e2 = build_scheme(F, mem, scheme, use_max=25)
    for _ in range(200):
        info = e2.run(max_attempts=1, sync_every=1, use_graph=True)
        torch.cuda.synchronize()
        if info["active"] == 0:
            break
    e3 = build_scheme(F, mem, scheme, use_max=25)
    for _ in range(30):   # more attempts than any member needs: finished ones idle
        e3.step(attempts=4, use_graph=True)
    e3.run(max_attempts=1, sync_every=1, use_graph=True)
    for i in range(len(mem)):
        a, ka, ma = ref.member(i)
        for e in (e2, e3):
            b, kb, mb = e.member(i)
            assert ma == mb, (i, ma, mb)
            assert np.array_equal(ka, kb) and torch.equal(a, b), i


def test_new_workspace_needs_reloaded_members(F):
    """A workspace set again holds no member: running refuses (FCH_E_INVALID)
    until every member is loaded into it, and then reaches the same states as
    an ensemble that never moved."""
    import ctypes as C
    log("ensemble workspace moved")
    mem = members_small()[:3]
    ref = build(F, mem, use_max=15)
    ref.run(max_attempts=500, sync_every=5, use_graph=True)
    ens = build(F, mem, use_max=15)
    nbytes = F.lib().fch_ensemble_workspace_bytes(ens.h)
    ws2 = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-ws2.data_ptr()) % 256
    assert F.lib().fch_ensemble_set_workspace(ens.h, C.c_void_p(ws2.data_ptr() + off),
                                              nbytes) == F.FCH_OK
    ens.ws = ws2
    with pytest.raises(F.FchError) as ei:
        ens.run(max_attempts=5, sync_every=5, use_graph=True)
    assert ei.value.code == F.FCH_E_INVALID
    for i, m in enumerate(mem):
        ens.load(i, torch.from_numpy(initial(m, seed=10 + i)).cuda())
    ens.run(max_attempts=500, sync_every=5, use_graph=True)
    for i in range(len(mem)):
        a, ka, ma = ens.member(i)
        b, kb, mb = ref.member(i)
        assert ma == mb and np.array_equal(ka, kb) and torch.equal(a, b), i


@pytest.mark.parametrize("scheme", ["imex", "sav"])
def test_adaptive_512_step_sequence_matches_oracle_controller(F, orc, scheme):
    """The 512^2 workload (six perturbed circles, eps 0.05) run adaptively to
    t = 0.01 at sigma_tol 1e-5 from k_first = 1e-9: the device-controlled
    attempts accept the same steps as the oracle's steppers driven by the
    oracle's own AM3 estimate and Sec. 3.2 controller, and end on the same
    state (and, for SAV, the same r)."""
    log("adaptive 512^2 %s step sequence vs the oracle controller" % scheme)
    kw, u0 = inputs.workload("c2")
    ens = F.Ensemble([kw], adapt=F.AdaptOpts(sigma_tol=1e-5), t_end=0.01, max_steps=100000,
                     k_first=1e-9, scheme=scheme)
    ens.load(0, torch.from_numpy(u0).cuda())
    ens.run(max_attempts=100000, sync_every=100, use_graph=True)
    uh, klog, mi = ens.member(0)
    z, d0 = F.sav_constants(F.fch_params(*[dict(kw, p=kw.get("p", 1), q=kw.get("q", 0.0),
                                                gamma_w=kw.get("gamma_w", 0.3),
                                                b_minus=-1.0, b_plus=1.0, beta1=2.0,
                                                beta2=1.0, zeta=0.0, D0=0.0)[k]
                                           for k, _ in F.fch_params._fields_]))
    m = orc.Model(**dict(kw, zeta=z, D0=d0))
    prev = orc.r2c(u0)
    if scheme == "sav":
        r_prev = float(np.sqrt(orc.E1(m, prev) + m.D0))
        cur, r_cur = orc.sav_step(m, prev, None, r_prev, r_prev, 1e-9, -1.0)
    else:
        cur = orc.imex_step(m, prev, None, 1e-9, -1.0)
    Fm, Fn = orc.F(m, prev), orc.F(m, cur)
    ks, t, kn, kt = [1e-9], 1e-9, 1e-9, 1e-9
    while t < 0.01 * (1 - 1e-14):
        kt = min(kt, 0.01 - t)
        if scheme == "sav":
            trial, r_trial = orc.sav_step(m, cur, prev, r_cur, r_prev, kt, kn)
        else:
            trial = orc.imex_step(m, cur, prev, kt, kn)
        Ft = orc.F(m, trial)
        e = orc.am3_error(m, trial, cur, Ft, Fn, Fm, kt, kn)
        ok, knext = orc.adapt_decide(e, kt, 1e-5, 1e-9, float("inf"))
        if ok:
            prev, cur, Fm, Fn = cur, trial, Fn, Ft
            if scheme == "sav":
                r_prev, r_cur = r_cur, r_trial
            t, kn = t + kt, kt
            ks.append(kt)
        kt = knext
    assert mi["accepted"] == len(ks) and len(klog) == len(ks)
    # k_next ~ e^(-1/3), and the estimate e (about sigma_tol) is a difference
    # of nearby states: a state difference of 1e-12 relative moves k by about
    # 1e-12 / (3 sigma_tol) ~ 3e-8.  Measured over the 181 steps: 3.0e-10
    # (IMEX) and 1.2e-8 (SAV).
    dk = float(np.max(np.abs(np.asarray(klog) / np.asarray(ks) - 1)))
    e_state = rel(uh.cpu().numpy().T, cur)
    log("  %d accepted steps; max |k_gpu/k_oracle - 1| = %.3e, state rel %.3e"
        % (len(ks), dk, e_state))
    assert dk < 1e-7, dk
    assert abs(mi["t"] - t) < 1e-12
    assert e_state < 1e-8
    if scheme == "sav":
        assert abs(mi["r_n"] - r_cur) < 1e-9 * abs(r_cur)
        assert abs(mi["r_nm1"] - r_prev) < 1e-9 * abs(r_prev)
