"""GPU parity: every C-ABI call against the CPU oracle on identical seeded
inputs.  Tolerances (relative L2 unless stated): transforms 1e-13, chemical
potential 1e-12, one step 1e-10, fixed-step trajectories 1e-8, SAV scalar
1e-12.  Spectra cross the boundary in the library's kx-major layout; the
tests transpose to the oracle's numpy layout."""
import json
import os
import sys

import numpy as np
import pytest
import torch

from paper_2006_04784_amd import inputs

pytestmark = pytest.mark.gpu

SIZES = [16, 32, 64, 128, 256, 512, 1024, 2048]


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_04784_amd import fch
    fch.lib()   # raises if the HIP library is missing
    return fch


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(uh_np):
    return torch.from_numpy(np.ascontiguousarray(uh_np.T)).to("cuda")


def host(uh_t):
    return uh_t.cpu().numpy().T


def model_kw(N, L, eps=0.1, q=0.0, eta1=1.45, eta2=2.0):
    return dict(N=N, L=L, eps=eps, eta1=eta1, eta2=eta2, p=1, q=q, zeta=1.1,
                D0=L * L * 1.05)


def pair(F, orc, **kw):
    return F.Plan(**kw), orc.Model(**kw)


# ---- transforms -------------------------------------------------------------
@pytest.mark.parametrize("N", SIZES)
def test_forward_inverse(F, orc, N):
    log("forward/inverse N=%d" % N)
    plan = F.Plan(**model_kw(N, 4 * np.pi))
    u = inputs.white_noise(N, seed=N)
    ref = orc.r2c(u)
    ut = torch.from_numpy(u).to("cuda")
    uh = plan.forward(ut)
    assert rel(host(uh), ref) < 1e-13
    back = plan.inverse(uh).cpu().numpy()
    assert rel(back, u) < 1e-13
    # inverse of a non-Hermitian spectrum: real part of the inverse DFT of the
    # Hermitian extension
    rng = np.random.default_rng(N)
    vh = ref + 0.05 * np.abs(ref).mean() * (rng.standard_normal(ref.shape)
                                            + 1j * rng.standard_normal(ref.shape))
    assert rel(plan.inverse(dev(vh)).cpu().numpy(), orc.c2r(vh)) < 1e-13
    st = plan.stats()
    assert st["fft_calls"] == 3


@pytest.mark.parametrize("N,B", [(16, 5), (64, 3), (256, 3), (1024, 2), (2048, 2)])
def test_batched_transforms(F, orc, N, B):
    """fch_forward_batch / fch_inverse_batch: each field equals the
    single-field transform bit for bit, the input spectra are left unchanged,
    and (N <= 256) the spectra match the oracle's DFT."""
    log("batched transforms N=%d B=%d" % (N, B))
    plan = F.Plan(**model_kw(N, 4 * np.pi))
    U = torch.stack([torch.from_numpy(inputs.white_noise(N, seed=100 + b)) for b in range(B)]).cuda()
    Uh = plan.forward_batch(U)
    for b in range(B):
        assert torch.equal(Uh[b], plan.forward(U[b].contiguous())), b
    if N <= 256:
        for b in range(B):
            ref = orc.r2c(U[b].cpu().numpy())
            assert rel(host(Uh[b]), ref) < 1e-13
    keep = Uh.clone()
    V = plan.inverse_batch(Uh)
    assert torch.equal(Uh, keep)
    for b in range(B):
        assert torch.equal(V[b], plan.inverse(Uh[b].contiguous())), b
    assert float((V - U).abs().max()) < 1e-12 * float(U.abs().max())
    with pytest.raises(RuntimeError):
        plan.inverse_batch(Uh, ws=torch.empty(16, dtype=torch.uint8, device="cuda"))


# ---- chemical potential -------------------------------------------------------
@pytest.mark.parametrize("N,q", [(16, 0.0), (64, 0.0), (64, 0.2), (256, 0.5), (512, 0.0)])
def test_chem_potential_and_energy(F, orc, N, q):
    log("chem potential N=%d q=%g" % (N, q))
    kw = model_kw(N, N * 4 * np.pi / 256 if N >= 64 else 2 * np.pi, q=q)
    plan, m = pair(F, orc, **kw)
    u = inputs.circle_bilayer(N, kw["L"], kw["eps"], seed=1)
    uh = orc.r2c(u)
    mu, E = plan.chem_potential(dev(uh), energy=True)
    ref = orc.mu(m, uh)
    assert rel(host(mu), ref) < 1e-12
    assert abs(E - orc.energy(m, uh)) < 1e-12 * max(1.0, abs(E))
    Fh = plan.rhs(dev(uh))
    assert rel(host(Fh), orc.F(m, uh)) < 1e-11


def test_chem_potential_dev(F, orc):
    """fch_chem_potential_dev gives fch_chem_potential's spectrum and energy bit
    for bit, mu on the grid equal to the inverse transform of that spectrum
    (and to the oracle's mu to 1e-12), and the same again when captured into a
    graph and replayed on a new state."""
    log("chem potential, device outputs")
    N = 128
    kw = model_kw(N, N * 4 * np.pi / 256, q=0.2)
    plan, m = pair(F, orc, **kw)
    uh = orc.r2c(inputs.circle_bilayer(N, kw["L"], kw["eps"], seed=1))
    uh2 = orc.r2c(inputs.circle_bilayer(N, kw["L"], kw["eps"], seed=2))
    x = dev(uh)
    mu_ref, E_ref = plan.chem_potential(x, energy=True)
    mud, mphys = plan.spec(), torch.empty((N, N), dtype=torch.float64, device="cuda")
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    plan.chem_potential_dev(x, mud, mphys, e, st)
    torch.cuda.synchronize()
    assert torch.equal(mud, mu_ref) and float(e.item()) == E_ref and int(st.item()) == 0
    assert torch.equal(mphys, plan.inverse(mud))
    ref_phys = orc.c2r(orc.mu(m, uh))
    assert rel(mphys.cpu().numpy(), ref_phys) < 1e-12
    with pytest.raises(F.FchError):
        plan.chem_potential_dev(x, x)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.chem_potential_dev(x, mud, mphys, e, st)
    x.copy_(dev(uh2))
    e.zero_()
    g.replay()
    torch.cuda.synchronize()
    mu2, E2 = plan.chem_potential(dev(uh2), energy=True)
    assert torch.equal(mud, mu2) and float(e.item()) == E2
    assert torch.equal(mphys, plan.inverse(mu2))


# ---- IMEX -------------------------------------------------------------------
def _c1(orc, F):
    kw, u0 = inputs.workload("c1")
    kw = dict(kw, zeta=1.1, D0=163.0)
    return F.Plan(**kw), orc.Model(**kw), orc.r2c(u0)


def test_imex_one_step_and_startup(F, orc):
    log("imex one step c1")
    plan, m, uh0 = _c1(orc, F)
    k = 1e-3
    u1_ref = orc.imex_step(m, uh0, None, k, -1.0)
    u1 = plan.step_imex(dev(uh0), None, k, -1.0)
    assert rel(host(u1), u1_ref) < 1e-10
    u2_ref = orc.imex_step(m, u1_ref, uh0, 1.7 * k, k)
    u2 = plan.step_imex(dev(u1_ref), dev(uh0), 1.7 * k, k)
    assert rel(host(u2), u2_ref) < 1e-10
    # output may alias u^{n-1}
    a, b = dev(u1_ref), dev(uh0)
    plan.step_imex(a, b, 1.7 * k, k, out=b)
    assert rel(host(b), u2_ref) < 1e-10


@pytest.mark.parametrize("beta", [(1.0, 2.0), (2.75, 0.25)])
def test_imex_stabilized_family(F, orc, beta):
    """IMEX with the stabilized L_0(beta) of eq. e:SAV-L0 (Figure Find-Beta's
    family) against the oracle: one step and a 50-step trajectory."""
    log("imex beta=%s c1" % (beta,))
    kw, u0 = inputs.workload("c1")
    kw = dict(kw, zeta=1.1, D0=163.0, beta1=beta[0], beta2=beta[1])
    plan, m = pair(F, orc, **kw)
    uh0 = orc.r2c(u0)
    u1_ref = orc.imex_step(m, uh0, None, 1e-3, -1.0)
    u2_ref = orc.imex_step(m, u1_ref, uh0, 1.5e-3, 1e-3)
    u2 = plan.step_imex(dev(u1_ref), dev(uh0), 1.5e-3, 1e-3)
    assert rel(host(u2), u2_ref) < 1e-10
    ref = orc.run_fixed(m, "imex", uh0, 1e-3, 50)
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    plan.run(a, b, scheme="imex", nsteps=50, k=1e-3)
    assert rel(host(a), ref) < 1e-8


def test_imex_trajectory_c1_200_steps(F, orc):
    log("imex trajectory c1 200 steps")
    plan, m, uh0 = _c1(orc, F)
    ref = orc.run_fixed(m, "imex", uh0, 1e-3, 200)
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    info = plan.run(a, b, scheme="imex", nsteps=200, k=1e-3)
    assert info["accepted"] == 200
    assert rel(host(a), ref) < 1e-8
    # mean (zero mode) conserved
    assert abs(host(a)[0, 0] - uh0[0, 0]) < 1e-13 * abs(uh0[0, 0]) * 64


def test_imex_full_size_fused_chain(F, orc):
    """1024^2 (the measured workload) in the fused launch sequence the
    benchmark times, three steps after the startup step."""
    log("imex 1024^2 fused chain")
    kw, u0 = inputs.workload("m1")
    kw = dict(kw, zeta=1.1, D0=kw["L"] ** 2 * 1.05)
    plan, m = pair(F, orc, **kw)
    uh0 = orc.r2c(u0)
    ref = orc.run_fixed(m, "imex", uh0, 1e-3, 4)
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    plan.run(a, b, scheme="imex", nsteps=4, k=1e-3)
    assert rel(host(a), ref) < 1e-10


def test_graph_replay_is_bit_identical(F, orc):
    """fch_plan_set_graph: the replayed fused chain equals the launched one
    bit for bit, including a remainder shorter than one replay and a second
    buffer pair (a new graph), and stays on the oracle."""
    log("imex graph replay c1")
    plan, m, uh0 = _c1(orc, F)
    with pytest.raises(RuntimeError):
        plan.set_graph(3)
    ref = orc.run_fixed(m, "imex", uh0, 1e-3, 37)
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    plan.run(a, b, scheme="imex", nsteps=37, k=1e-3)
    plan.set_graph(8)
    for rep in range(2):
        c, d = dev(uh0), torch.zeros_like(dev(uh0))
        info = plan.run(c, d, scheme="imex", nsteps=37, k=1e-3)
        assert info["accepted"] == 37
        assert torch.equal(c, a) and torch.equal(d, b), rep
    assert rel(host(c), ref) < 1e-8
    # continuing without startup on the same pair reuses the graph
    plan.run(a, b, scheme="imex", nsteps=20, k=1e-3, k_prev=1e-3, startup=False)
    plan.set_graph(0)
    plan.run(c, d, scheme="imex", nsteps=20, k=1e-3, k_prev=1e-3, startup=False)
    assert torch.equal(c, a) and torch.equal(d, b)


def test_graph_replay_full_size(F, orc):
    """1024^2 with graph replay as the benchmark runs it: equal to the
    launched chain bit for bit and to the oracle after 4 steps."""
    log("imex 1024^2 graph replay")
    kw, u0 = inputs.workload("m1")
    kw = dict(kw, zeta=1.1, D0=kw["L"] ** 2 * 1.05)
    plan, m = pair(F, orc, **kw)
    uh0 = orc.r2c(u0)
    ref = orc.run_fixed(m, "imex", uh0, 1e-3, 4)
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    plan.set_graph(2)
    plan.run(a, b, scheme="imex", nsteps=4, k=1e-3)
    assert rel(host(a), ref) < 1e-10
    plan.set_graph(16)
    plan.run(a, b, scheme="imex", nsteps=40, k=1e-3, k_prev=1e-3, startup=False)
    plan.set_graph(0)
    c, d = dev(uh0), torch.zeros_like(dev(uh0))
    plan.run(c, d, scheme="imex", nsteps=4, k=1e-3)
    plan.run(c, d, scheme="imex", nsteps=40, k=1e-3, k_prev=1e-3, startup=False)
    assert torch.equal(c, a) and torch.equal(d, b)


# ---- SAV --------------------------------------------------------------------
def test_sav_step_and_r(F, orc):
    log("sav step c1")
    plan, m, uh0 = _c1(orc, F)
    k = 1e-3
    r0_ref = float(np.sqrt(orc.E1(m, uh0) + m.D0))
    r0 = plan.sav_r(dev(uh0))
    assert abs(r0 - r0_ref) < 1e-12 * r0_ref
    u1_ref, r1_ref = orc.sav_step(m, uh0, None, r0_ref, r0_ref, k, -1.0)
    u1, r1 = plan.step_sav(dev(uh0), None, r0_ref, r0_ref, k, -1.0)
    assert rel(host(u1), u1_ref) < 1e-10
    assert abs(r1 - r1_ref) < 1e-12 * abs(r1_ref)
    u2_ref, r2_ref = orc.sav_step(m, u1_ref, uh0, 1.01 * r1_ref, r0_ref, 1.3 * k, k)
    u2, r2 = plan.step_sav(dev(u1_ref), dev(uh0), 1.01 * r1_ref, r0_ref, 1.3 * k, k)
    assert rel(host(u2), u2_ref) < 1e-10
    assert abs(r2 - r2_ref) < 1e-12 * abs(r2_ref)
    # deterministic reductions: bitwise repeatable
    u2b, r2b = plan.step_sav(dev(u1_ref), dev(uh0), 1.01 * r1_ref, r0_ref, 1.3 * k, k)
    assert r2b == r2 and torch.equal(u2b, u2)


def test_sav_trajectory(F, orc):
    log("sav trajectory c1 60 steps")
    plan, m, uh0 = _c1(orc, F)
    ref, states = orc.run_fixed(m, "sav", uh0, 1e-3, 60, record=True)
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    info = plan.run(a, b, scheme="sav", nsteps=60, k=1e-3)
    assert rel(host(a), ref) < 1e-8
    assert rel(host(b), states[-2]) < 1e-8


def test_sav_fused_chain(F, orc):
    """fch_run's fixed-step SAV chain keeps r on the device (the column pass
    after each SAV step solves for r^{n+1} in every workgroup and starts the
    next step); it matches a loop of fch_step_sav calls and the oracle's
    states and scalars."""
    log("sav fused chain c1 40 steps")
    plan, m, uh0 = _c1(orc, F)
    k = 1e-3
    r0 = float(np.sqrt(orc.E1(m, uh0) + m.D0))
    o_m, o_n = None, uh0
    rm = rn = r0
    for i in range(40):
        new, rnew = orc.sav_step(m, o_n, o_m, rn, rm, k, -1.0 if i == 0 else k)
        o_m, o_n = o_n, new
        rm, rn = rn, rnew
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    info = plan.run(a, b, scheme="sav", nsteps=40, k=k)
    assert rel(host(a), o_n) < 1e-8 and rel(host(b), o_m) < 1e-8
    assert abs(info["rs"][0] - rn) < 1e-10 * abs(rn)
    assert abs(info["rs"][1] - rm) < 1e-10 * abs(rm)
    # the same steps one call at a time
    x, y = dev(uh0), None
    qn = qm = plan.sav_r(dev(uh0))
    for i in range(40):
        z, qnew = plan.step_sav(x, y if y is not None else x, qn, qm, k, -1.0 if i == 0 else k)
        y, x = x, z
        qm, qn = qn, qnew
    assert rel(host(a), host(x)) < 1e-13 and rel(host(b), host(y)) < 1e-13
    assert abs(info["rs"][0] - qn) < 1e-13 * abs(qn) and abs(info["rs"][1] - qm) < 1e-13 * abs(qm)
    # continuing a run (rs in/out, k_prev = k) equals one longer run
    a2, b2 = dev(uh0), torch.zeros_like(dev(uh0))
    i1 = plan.run(a2, b2, scheme="sav", nsteps=25, k=k)
    i2 = plan.run(a2, b2, scheme="sav", nsteps=15, k=k, k_prev=k, startup=False, rs=i1["rs"])
    assert rel(host(a2), host(a)) < 1e-13
    assert abs(i2["rs"][0] - info["rs"][0]) < 1e-13 * abs(info["rs"][0])


# ---- PSD --------------------------------------------------------------------
def test_psd_fixed_iterations_and_converged(F, orc):
    log("psd c1")
    plan, m, uh0 = _c1(orc, F)
    k = 1e-3
    u1 = orc.imex_step(m, uh0, None, k, -1.0)
    ref, it, _, rc = orc.psd_step(m, u1, uh0, k, k, fixed_iters=5)
    out, st = plan.step_psd(dev(u1), dev(uh0), k, k, fixed_iters=5)
    assert st["iters"] == 5
    assert rel(host(out), ref) < 1e-10
    # converged solve: replay the GPU's iteration count on the oracle
    out, st = plan.step_psd(dev(u1), dev(uh0), k, k, tol=1e-10)
    assert st["last_ratio"] < 1e-10
    ref, it, ratio, rc = orc.psd_step(m, u1, uh0, k, k, fixed_iters=st["iters"])
    assert rel(host(out), ref) < 1e-10
    # the oracle's own stopping decision agrees within one iteration
    _, it2, _, _ = orc.psd_step(m, u1, uh0, k, k, tol=1e-10)
    assert abs(it2 - st["iters"]) <= 1
    # a guess: projected to the mean of u^n
    guess = u1.copy()
    guess[0, 0] += 5.0
    out, st = plan.step_psd(dev(u1), dev(uh0), k, k, guess=dev(guess), fixed_iters=3)
    ref, _, _, _ = orc.psd_step(m, u1, uh0, k, k, guess=guess, fixed_iters=3)
    assert rel(host(out), ref) < 1e-10


def test_psd_noconv(F, orc):
    plan, m, uh0 = _c1(orc, F)
    u1 = orc.imex_step(m, uh0, None, 1e-3, -1.0)
    out, st = plan.step_psd(dev(u1), dev(uh0), 1e-3, 1e-3, tol=1e-30, max_iter=6,
                            raise_noconv=False)
    assert st["status"] == F.FCH_E_NOCONV and st["iters"] == 6
    ref, _, _, _ = orc.psd_step(m, u1, uh0, 1e-3, 1e-3, fixed_iters=6)
    assert rel(host(out), ref) < 1e-10


def test_psd_full_size_2048(F, orc):
    log("psd 2048^2, 2 fixed iterations")
    N, L, eps = 2048, 16 * np.pi, 0.05
    kw = dict(model_kw(N, L, eps=eps))
    plan, m = pair(F, orc, **kw)
    u0 = inputs.circle_bilayer(N, L, eps, seed=3, noise=1e-3)
    uh0 = orc.r2c(u0)
    u1 = orc.imex_step(m, uh0, None, 1e-4, -1.0)
    ref, _, _, _ = orc.psd_step(m, u1, uh0, 1e-4, 1e-4, fixed_iters=2)
    out, st = plan.step_psd(dev(u1), dev(uh0), 1e-4, 1e-4, fixed_iters=2)
    assert rel(host(out), ref) < 1e-10


# ---- adaptivity -------------------------------------------------------------
def test_adapt_dt_matches_oracle(F, orc):
    log("adapt_dt c1")
    plan, m, uh0 = _c1(orc, F)
    k0 = 1e-4
    u1 = orc.imex_step(m, uh0, None, k0, -1.0)
    F0, F1 = orc.F(m, uh0), orc.F(m, u1)
    for kt in (1e-4, 5e-4, 4e-3):
        ut = orc.imex_step(m, u1, uh0, kt, k0)
        e_ref = orc.am3_error(m, ut, u1, orc.F(m, ut), F1, F0, kt, k0)
        acc_ref, kn_ref = orc.adapt_decide(e_ref, kt, 1e-5, 1e-9, np.inf)
        Ft, acc, kn, e = plan.adapt_dt(dev(ut), dev(u1), dev(F1), dev(F0), kt, k0,
                                       F.AdaptOpts(sigma_tol=1e-5))
        assert abs(e - e_ref) < 1e-9 * e_ref
        if abs(e_ref - 1e-5) / 1e-5 > 1e-9:
            assert acc == acc_ref
        assert abs(kn - kn_ref) < 1e-9 * kn_ref
        assert rel(host(Ft), orc.F(m, ut)) < 1e-11


def test_adaptive_run_replayed_by_oracle(F, orc):
    """The GPU adaptive IMEX run is replayed on the oracle with the GPU's
    accepted step sizes; decisions are re-derived by the oracle."""
    log("adaptive imex c1 replay")
    plan, m, uh0 = _c1(orc, F)
    opts = F.AdaptOpts(sigma_tol=1e-5)
    k1 = 1e-9
    cur = plan.step_imex(dev(uh0), None, k1, -1.0)
    prev = dev(uh0)
    Fn, Fm = plan.rhs(cur), plan.rhs(prev)
    kn, kt, t = k1, k1, k1
    sched = [k1]
    for _ in range(40):
        trial = plan.step_imex(cur, prev, kt, kn)
        Ft, acc, knext, e = plan.adapt_dt(trial, cur, Fn, Fm, kt, kn, opts)
        if acc:
            prev, cur = cur, trial
            Fm, Fn = Fn, Ft
            t += kt
            kn = kt
            sched.append(kt)
        kt = knext
    # oracle replay of the accepted schedule
    o_prev, o_cur = uh0, orc.imex_step(m, uh0, None, sched[0], -1.0)
    o_Fm, o_Fn = orc.F(m, o_prev), orc.F(m, o_cur)
    for i in range(1, len(sched)):
        nxt = orc.imex_step(m, o_cur, o_prev, sched[i], sched[i - 1])
        e = orc.am3_error(m, nxt, o_cur, orc.F(m, nxt), o_Fn, o_Fm, sched[i], sched[i - 1])
        acc, _ = orc.adapt_decide(e, sched[i], 1e-5, 1e-9, np.inf)
        assert acc or abs(e - 1e-5) / 1e-5 < 1e-9
        o_prev, o_cur = o_cur, nxt
        o_Fm, o_Fn = o_Fn, orc.F(m, nxt)
    assert len(sched) > 10 and sched[-1] > 100 * k1
    assert rel(host(cur), o_cur) < 1e-8
    # the library's own adaptive driver takes the same decisions
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    info = plan.run(a, b, scheme="imex", adaptive=True, startup=True, t_end=t, k_first=k1,
                    adapt=opts, nsteps=len(sched))
    assert info["accepted"] == len(sched)
    assert rel(host(a), host(cur)) < 1e-12


# ---- edge cases ----------------------------------------------------------------
def test_invalid_arguments(F, orc):
    plan, m, uh0 = _c1(orc, F)
    x = dev(uh0)
    with pytest.raises(F.FchError) as ei:
        plan.step_imex(x, None, -1e-3, -1.0)
    assert ei.value.code == F.FCH_E_INVALID
    with pytest.raises(F.FchError):
        plan.step_imex(x, None, 1e-3, 1e-3)      # k_n > 0 needs u^{n-1}
    with pytest.raises(F.FchError):
        plan.step_imex(x, x, 1e-3, 1e-3, out=x)  # output aliases u^n
    with pytest.raises(ValueError):
        plan.forward(torch.zeros((64, 63), dtype=torch.float64, device="cuda"))


def test_nonfinite_detected(F, orc):
    plan, m, uh0 = _c1(orc, F)
    bad = uh0.copy()
    bad[3, 2] = np.nan
    with pytest.raises(F.FchError) as ei:
        plan.chem_potential(dev(bad), energy=True)
    assert ei.value.code == F.FCH_E_NONFINITE
    with pytest.raises(F.FchError) as ei:
        plan.step_sav(dev(bad), None, 1.0, 1.0, 1e-3, -1.0)
    assert ei.value.code == F.FCH_E_NONFINITE
    # the plan recovers on clean input
    mu = plan.chem_potential(dev(uh0))
    assert rel(host(mu), orc.mu(m, uh0)) < 1e-12


def test_sav_rejects_negative_shift(F, orc):
    kw, u0 = inputs.workload("c1")
    kw = dict(kw, zeta=1.1, D0=-1e6)
    plan = F.Plan(**kw)
    uh0 = orc.r2c(u0)
    with pytest.raises(F.FchError) as ei:
        plan.step_sav(dev(uh0), None, 1.0, 1.0, 1e-3, -1.0)
    assert ei.value.code == F.FCH_E_INVALID


def test_long_trajectory_256_stays_on_oracle(F, orc):
    """600 fixed steps at 256^2 (h/eps = 0.49): a non-real component in the
    kx = 0 and kx = N/2 columns, seeded by rounding and amplified by the
    explicit linear terms, once drove the GPU state off the oracle here."""
    log("imex 256^2, 600 steps")
    N, L = 256, 4 * np.pi
    kw = model_kw(N, L)
    plan, m = pair(F, orc, **kw)
    uh0 = orc.r2c(inputs.circle_bilayer(N, L, 0.1, seed=0))
    ref = orc.run_fixed(m, "imex", uh0, 1e-3, 600)
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    plan.run(a, b, scheme="imex", nsteps=600, k=1e-3)
    assert rel(host(a), ref) < 1e-8
    # every state the library writes is the spectrum of a real field
    for col in (0, N // 2):
        c = a[col].cpu().numpy()
        assert np.array_equal(c, np.conj(c[(-np.arange(N)) % N]))


@pytest.mark.parametrize("N", [16, 64, 256, 512, 1024, 2048])
def test_every_launch_variant(F, orc, N):
    """Each compiled row-pass and column-pass variant gives the oracle's
    transforms, IMEX step, ETDRK2 step, SAV step (row partial sums) and PSD
    solve (the row pass's stopping test; the oracle replays the iteration count)."""
    log("launch variants N=%d" % N)
    rows, cols = F.config_list(N)
    L = N * 4 * np.pi / 256
    kw = model_kw(N, L)
    plan, m = pair(F, orc, **kw)
    u0 = inputs.circle_bilayer(N, L, 0.1, seed=2)
    uh0 = orc.r2c(u0)
    u1 = orc.imex_step(m, uh0, None, 1e-3, -1.0)
    ref = orc.imex_step(m, u1, uh0, 1e-3, 1e-3)
    ref_etd = orc.etd_step(m, u1, 1e-3)
    r0 = float(np.sqrt(orc.E1(m, uh0) + m.D0))
    ref_sav, ref_r = orc.sav_step(m, u1, uh0, r0, r0, 1e-3, 1e-3)
    psd_ref = {}
    for i in range(max(len(rows), len(cols))):
        r, c = rows[i % len(rows)], cols[i % len(cols)]
        plan.set_config((r[0], r[1], r[2], c[0], c[1]))
        assert plan.get_config() == (r[0], r[1], r[2], c[0], c[1])
        uh = plan.forward(torch.from_numpy(u0).cuda())
        assert rel(host(uh), uh0) < 1e-13, (r, c)
        assert rel(plan.inverse(uh).cpu().numpy(), u0) < 1e-13, (r, c)
        out = plan.step_imex(dev(u1), dev(uh0), 1e-3, 1e-3)
        assert rel(host(out), ref) < 1e-10, (r, c)
        a, b = dev(u1), dev(uh0)
        plan.run(a, b, scheme="imex", nsteps=1, k=1e-3, k_prev=1e-3, startup=False)
        assert rel(host(a), ref) < 1e-10, (r, c)
        assert rel(host(plan.step_etd(dev(u1), 1e-3)), ref_etd) < 1e-10, (r, c)
        out, r1 = plan.step_sav(dev(u1), dev(uh0), r0, r0, 1e-3, 1e-3)
        assert rel(host(out), ref_sav) < 1e-10 and abs(r1 - ref_r) < 1e-12 * abs(ref_r), (r, c)
        out, st = plan.step_psd(dev(u1), dev(uh0), 1e-3, 1e-3, tol=1e-10)
        it = st["iters"]
        if it not in psd_ref:
            psd_ref[it] = orc.psd_step(m, u1, uh0, 1e-3, 1e-3, fixed_iters=it)[0]
        assert rel(host(out), psd_ref[it]) < 1e-10, (r, c, it)


def test_autotune_picks_a_compiled_variant(F, orc):
    log("autotune 256")
    N, L = 256, 4 * np.pi
    plan, m = pair(F, orc, **model_kw(N, L))
    uh0 = orc.r2c(inputs.circle_bilayer(N, L, 0.1, seed=0))
    u1 = orc.imex_step(m, uh0, None, 1e-3, -1.0)
    a, b = dev(u1), dev(uh0)
    a0, b0 = a.clone(), b.clone()
    cfg, us = plan.autotune(a, b, k=1e-3, reps=3)
    rows, cols = F.config_list(N)
    assert cfg[:3] in rows and cfg[3:] in cols and us[0] > 0 and us[1] > 0
    assert torch.equal(a, a0) and torch.equal(b, b0)     # inputs untouched
    out = plan.step_imex(a, b, 1e-3, 1e-3)
    assert rel(host(out), orc.imex_step(m, u1, uh0, 1e-3, 1e-3)) < 1e-10


def test_autotune_cache(F, orc, tmp_path):
    """A tuned choice is kept in a JSON cache keyed by architecture, N and the
    library: a second plan takes it from the file without timing (the plan's
    configuration is set, the file unchanged); another N adds an entry; an
    unreadable file counts as empty."""
    log("autotune cache")
    cache = str(tmp_path / "tune.json")
    N, L = 256, 4 * np.pi
    plan = F.Plan(**model_kw(N, L))
    a = plan.forward(torch.from_numpy(inputs.circle_bilayer(N, L, 0.1, seed=0)).cuda())
    b = a.clone()
    cfg, us = plan.autotune(a, b, reps=2, cache=cache)
    key = F.tune_key(N)
    d = json.load(open(cache))
    assert d[key]["config"] == list(cfg)
    mtime = os.path.getmtime(cache)
    plan2 = F.Plan(**model_kw(N, L))
    plan2.set_config(None)
    cfg2, us2 = plan2.autotune(a, b, reps=2, cache=cache)
    assert cfg2 == cfg and tuple(us2) == tuple(us) and plan2.get_config() == cfg
    assert os.path.getmtime(cache) == mtime
    plan3 = F.Plan(**model_kw(128, 2 * np.pi))
    a3 = plan3.forward(torch.from_numpy(inputs.circle_bilayer(128, 2 * np.pi, 0.1, seed=0)).cuda())
    plan3.autotune(a3, a3.clone(), reps=2, cache=cache)
    assert set(json.load(open(cache))) == {key, F.tune_key(128)}
    with open(cache, "w") as fh:
        fh.write("{not json")
    cfg4, _ = plan2.autotune(a, b, reps=2, cache=cache)
    assert list(json.load(open(cache))) == [key]


# ---- device-scalar (graph-capturable) steps ---------------------------------
def test_dev_steps_equal_host_steps(F, orc):
    """fch_step_imex_dev / _sav_dev / _psd_dev / _etd_dev / fch_adapt_dt_dev read
    their scalars from device memory and equal the host-scalar calls bit for bit."""
    log("device-scalar steps c1")
    plan, m, uh0 = _c1(orc, F)
    k = 1e-3
    d = lambda *v: torch.tensor(v, dtype=torch.float64, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    a0 = dev(uh0)
    # IMEX: startup, then a ratio change
    u1 = plan.step_imex(a0, None, k, -1.0)
    u1d = plan.step_imex_dev(a0, a0, d(k, -1.0), plan.spec(), st)
    assert torch.equal(u1, u1d) and int(st.item()) == 0
    u2 = plan.step_imex(u1, a0, 1.7 * k, k)
    u2d = plan.step_imex_dev(u1, a0, d(1.7 * k, k), plan.spec(), st)
    assert torch.equal(u2, u2d) and int(st.item()) == 0
    # SAV
    r0 = plan.sav_r(a0)
    s1, r1 = plan.step_sav(u1, a0, r0, r0, 1.7 * k, k)
    rn = torch.zeros(1, dtype=torch.float64, device="cuda")
    s1d = plan.step_sav_dev(u1, a0, d(r0, r0), d(1.7 * k, k), plan.spec(), rn, st)
    assert torch.equal(s1, s1d) and float(rn.item()) == r1 and int(st.item()) == 0
    # PSD (lambda from the table, and a fixed lambda)
    for lam in (0.0, 1.2):
        p1, info = plan.step_psd(u1, a0, 1.7 * k, k, tol=1e-10, lam=lam)
        it = torch.zeros(1, dtype=torch.int32, device="cuda")
        p1d = plan.step_psd_dev(u1, a0, d(1.7 * k, k), plan.spec(), it, st, tol=1e-10,
                                max_iter=200, lam=lam)
        assert torch.equal(p1, p1d) and int(it.item()) == info["iters"] and int(st.item()) == 0
    # adaptivity
    Fn, Fm = plan.rhs(u1), plan.rhs(a0)
    Ft, acc, kn, err = plan.adapt_dt(u2, u1, Fn, Fm, 1.7 * k, k)
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    Ftd = plan.adapt_dt_dev(u2, u1, Fn, Fm, d(1.7 * k, k), plan.spec(), out, st)
    o = out.cpu().numpy()
    assert torch.equal(Ft, Ftd) and o[0] == float(acc) and o[1] == kn and o[2] == err
    assert int(st.item()) == 0
    # ETDRK2, with and without a cached F(u^n)
    e1 = plan.step_etd(u1, 1.7 * k)
    e1d = plan.step_etd_dev(u1, d(1.7 * k), plan.spec(), status_dev=st)
    assert torch.equal(e1, e1d) and int(st.item()) == 0
    e2 = plan.step_etd(u1, 1.7 * k, F_n=Fn)
    e2d = plan.step_etd_dev(u1, d(1.7 * k), plan.spec(), F_n=Fn, status_dev=st)
    assert torch.equal(e2, e2d) and int(st.item()) == 0
    plan.step_etd_dev(u1, d(0.0), plan.spec(), status_dev=st)
    assert int(st.item()) == -1
    # invalid scalars are reported on the device
    plan.step_imex_dev(u1, a0, d(-1.0, k), plan.spec(), st)
    assert int(st.item()) == -1
    it = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    plan.step_psd_dev(u1, a0, d(float("nan"), k), plan.spec(), it, st, max_iter=5)
    assert int(st.item()) == -1 and int(it.item()) == 0
    plan.adapt_dt_dev(u2, u1, Fn, Fm, d(1.7 * k, 0.0), plan.spec(), out, st)
    assert int(st.item()) == -1
    # a PSD limit that is too small reports non-convergence
    plan.step_psd_dev(u1, a0, d(1.7 * k, k), plan.spec(), it, st, tol=1e-14, max_iter=2)
    assert int(st.item()) == -5 and int(it.item()) == 2


def test_dev_steps_in_a_captured_graph(F, orc):
    """Two device-scalar IMEX steps captured in a HIP graph (torch capture on
    the plan's stream), replayed with new inputs and step sizes written
    between replays: every replay equals the eager host-scalar steps."""
    log("device-scalar steps under graph capture")
    plan, m, uh0 = _c1(orc, F)
    k = 1e-3
    a0 = dev(uh0)
    u1 = plan.step_imex(a0, None, k, -1.0)
    x_nm1, x_n = a0.clone(), u1.clone()
    y1, y2 = plan.spec(), plan.spec()
    kd1 = torch.tensor([k, k], dtype=torch.float64, device="cuda")
    kd2 = torch.tensor([k, k], dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    # one eager call before capture
    plan.step_imex_dev(x_n, x_nm1, kd1, y1, st)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.step_imex_dev(x_n, x_nm1, kd1, y1, st)
        plan.step_imex_dev(y1, x_n, kd2, y2, st)
    cases = [(a0, u1, 1.3 * k, k, 0.8 * k), (u1, plan.step_imex(u1, a0, k, k), k, k, 2.0 * k),
             (a0, u1, 0.5 * k, k, 0.5 * k)]
    for rep, (um, un, k1, k0, k2) in enumerate(cases):
        x_nm1.copy_(um)
        x_n.copy_(un)
        kd1.copy_(torch.tensor([k1, k0], dtype=torch.float64))
        kd2.copy_(torch.tensor([k2, k1], dtype=torch.float64))
        g.replay()
        torch.cuda.synchronize()
        e1 = plan.step_imex(un, um, k1, k0)
        e2 = plan.step_imex(e1, un, k2, k1)
        assert torch.equal(y1, e1) and torch.equal(y2, e2), rep
        assert int(st.item()) == 0


def test_split_column_passes_captured_and_aliased(F, orc):
    """At 4096^2 the fused column passes run as two launches, the pair of
    self-conjugate columns on the plan's side stream (forked from and joined
    back to the plan's stream).  Captured into a graph with torch's capture of
    that stream, two device-scalar IMEX steps replay bit for bit like the eager
    steps; an aliased output (u^{n+1} over u^{n-1}) equals the plain call."""
    log("4096^2: split column passes under graph capture, aliasing")
    N, L = 4096, 64 * np.pi
    plan = F.Plan(**model_kw(N, L))
    k = 1e-3
    a0 = plan.forward(torch.from_numpy(inputs.circle_bilayer(N, L, 0.1, seed=5)).cuda())
    u1 = plan.step_imex(a0, None, k, -1.0)
    ref = plan.step_imex(u1, a0, 1.3 * k, k)
    b = a0.clone()
    plan.step_imex(u1, b, 1.3 * k, k, out=b)
    assert torch.equal(b, ref)
    x_nm1, x_n = a0.clone(), u1.clone()
    y1, y2 = plan.spec(), plan.spec()
    kd1 = torch.tensor([k, k], dtype=torch.float64, device="cuda")
    kd2 = torch.tensor([k, k], dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.step_imex_dev(x_n, x_nm1, kd1, y1, st)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.step_imex_dev(x_n, x_nm1, kd1, y1, st)
        plan.step_imex_dev(y1, x_n, kd2, y2, st)
    for rep, (um, un, k1, k0, k2) in enumerate([(a0, u1, 1.3 * k, k, 0.8 * k),
                                                (u1, ref, k, 1.3 * k, 2.0 * k)]):
        x_nm1.copy_(um)
        x_n.copy_(un)
        kd1.copy_(torch.tensor([k1, k0], dtype=torch.float64))
        kd2.copy_(torch.tensor([k2, k1], dtype=torch.float64))
        g.replay()
        torch.cuda.synchronize()
        e1 = plan.step_imex(un, um, k1, k0)
        e2 = plan.step_imex(e1, un, k2, k1)
        assert torch.equal(y1, e1) and torch.equal(y2, e2), rep
        assert int(st.item()) == 0


def test_output_aliasing_u_nm1_is_exact(F, orc):
    """IMEX, SAV and PSD with uh_np1 == uh_nm1 equal the non-aliased call bit
    for bit: every value a column workgroup reads (including the mirrored
    values of the self-conjugate columns kx = 0, N/2) is read before any
    output of that workgroup is written."""
    log("aliasing u^{n+1} = u^{n-1}")
    plan, m, uh0 = _c1(orc, F)
    k = 1e-3
    a0 = dev(uh0)
    u1 = plan.step_imex(a0, None, k, -1.0)
    ref = plan.step_imex(u1, a0, 1.3 * k, k)
    b = a0.clone()
    plan.step_imex(u1, b, 1.3 * k, k, out=b)
    assert torch.equal(b, ref)
    r0 = plan.sav_r(a0)
    ref, rr = plan.step_sav(u1, a0, r0, r0, 1.3 * k, k)
    b = a0.clone()
    _, rb = plan.step_sav(u1, b, r0, r0, 1.3 * k, k, out=b)
    assert torch.equal(b, ref) and rb == rr
    ref, st = plan.step_psd(u1, a0, 1.3 * k, k, tol=1e-10)
    b = a0.clone()
    _, st2 = plan.step_psd(u1, b, 1.3 * k, k, tol=1e-10, out=b)
    assert torch.equal(b, ref) and st2["iters"] == st["iters"]


def test_self_conjugate_columns_stay_exactly_hermitian(F, orc):
    """A state whose kx = 0 and N/2 columns are perturbed off Hermitian
    symmetry is stepped: the column pass uses their Hermitian parts, so every
    state it writes has U(ky) == conj U(N - ky) bit for bit in those columns,
    and the trajectory equals the oracle's from the projected start."""
    log("self-conjugate columns")
    plan, m, uh0 = _c1(orc, F)
    N = uh0.shape[0]
    rng = np.random.default_rng(5)
    bad = uh0.copy()
    for kx in (0, N // 2):
        bad[:, kx] += 1e-3 * (rng.normal(size=N) + 1j * rng.normal(size=N)) * np.abs(uh0[:, kx]).max()
    proj = bad.copy()
    for kx in (0, N // 2):
        col = bad[:, kx]
        proj[:, kx] = 0.5 * (col + np.conj(col[(-np.arange(N)) % N]))
    ref = orc.run_fixed(m, "imex", proj, 1e-3, 30)
    a, b = dev(bad), torch.zeros_like(dev(bad))
    plan.run(a, b, scheme="imex", nsteps=30, k=1e-3)
    h = host(a)
    for kx in (0, N // 2):
        col = h[:, kx]
        assert np.array_equal(col, np.conj(col[(-np.arange(N)) % N])), kx
    assert rel(h, ref) < 1e-8


def test_constant_state_is_a_fixed_point(F, orc):
    """Degenerate input: a spatially constant u has Lap u = 0 and a constant
    chemical potential, so F(u) = Lap mu = 0 and every scheme keeps it (the
    mean to rounding, every other mode at rounding level); the oracle agrees."""
    log("constant state")
    kw = model_kw(64, 4 * np.pi)
    plan, m = pair(F, orc, **kw)
    u = np.full((64, 64), -0.3)
    uh = orc.r2c(u)
    a = dev(uh)
    k = 1e-3
    mean = abs(uh[0, 0])

    def check(out, what):
        h = host(out)
        assert abs(h[0, 0] - uh[0, 0]) <= 1e-14 * mean, what
        rest = h.copy()
        rest[0, 0] = 0.0
        assert np.abs(rest).max() <= 1e-12 * mean, what

    check(plan.step_imex(a, None, k, -1.0), "imex startup")
    check(plan.step_imex(a, a, 1.5 * k, k), "imex")
    r0 = plan.sav_r(a)
    out, r1 = plan.step_sav(a, a, r0, r0, k, k)
    check(out, "sav")
    assert abs(r1 - r0) <= 1e-12 * abs(r0)
    out, st = plan.step_psd(a, a, k, k, tol=1e-10)
    check(out, "psd")
    assert st["iters"] <= 2
    F0 = plan.rhs(a)
    assert float(F0.abs().max()) <= 1e-10 * mean
    x, y = a.clone(), a.clone()
    info = plan.run(x, y, scheme="imex", adaptive=True, startup=True, t_end=0.05, k_first=1e-4)
    check(x, "adaptive")
    assert info["accepted"] >= 2
    ref = orc.imex_step(m, uh, uh, 1.5 * k, k)
    assert np.abs(ref - uh).max() <= 1e-12 * mean


def test_batch_limits(F, orc):
    plan = F.Plan(**model_kw(16, 2 * np.pi))
    lib = F.lib()
    U = torch.zeros((1, 16, 16), dtype=torch.float64, device="cuda")
    Uh = torch.zeros((1, 9, 16), dtype=torch.complex128, device="cuda")
    import ctypes as C
    for b in (0, 65536, -1):
        assert lib.fch_forward_batch(plan.h, b, C.c_void_p(U.data_ptr()),
                                     C.c_void_p(Uh.data_ptr())) == F.FCH_E_INVALID
    assert lib.fch_inverse_batch_ws_bytes(plan.h, 0) == 0
    assert lib.fch_inverse_batch_ws_bytes(plan.h, 3) == 3 * 16 * 9 * 16


def test_c2_adaptive_imex_and_sav_512(F, orc):
    """The 512^2 workload (eps 0.05, six perturbed bilayers): adaptive
    BDF2-IMEX and BDF2-SAV driven by the library (fch_step_*, fch_adapt_dt)
    for 40 accepted steps; the oracle replays the accepted step sizes and the
    states agree within the trajectory tolerance."""
    kw, u0 = inputs.workload("c2")
    kw = dict(kw, zeta=1.1, D0=kw["L"] ** 2 * 1.05)
    plan, m = pair(F, orc, **kw)
    uh0 = orc.r2c(u0)
    opts = F.AdaptOpts(sigma_tol=1e-5)
    k1 = 1e-6
    for scheme in ("imex", "sav"):
        log("c2 adaptive %s 512^2" % scheme)
        a0 = dev(uh0)
        r0 = plan.sav_r(a0) if scheme == "sav" else 0.0
        if scheme == "imex":
            cur = plan.step_imex(a0, None, k1, -1.0)
        else:
            cur, r1 = plan.step_sav(a0, None, r0, r0, k1, -1.0)
        prev = a0
        rs = (r1, r0) if scheme == "sav" else None
        Fn, Fm = plan.rhs(cur), plan.rhs(prev)
        kn, kt = k1, k1
        sched = [k1]
        while len(sched) < 41:
            if scheme == "imex":
                trial = plan.step_imex(cur, prev, kt, kn)
            else:
                trial, rt = plan.step_sav(cur, prev, rs[0], rs[1], kt, kn)
            Ft, acc, knext, e = plan.adapt_dt(trial, cur, Fn, Fm, kt, kn, opts)
            if acc:
                prev, cur = cur, trial
                Fm, Fn = Fn, Ft
                kn = kt
                sched.append(kt)
                if scheme == "sav":
                    rs = (rt, rs[0])
            kt = knext
        assert sched[-1] > 3 * k1
        # oracle replay of the accepted schedule
        if scheme == "imex":
            o_prev, o_cur = uh0, orc.imex_step(m, uh0, None, sched[0], -1.0)
            for i in range(1, len(sched)):
                o_prev, o_cur = o_cur, orc.imex_step(m, o_cur, o_prev, sched[i], sched[i - 1])
        else:
            ro = np.sqrt(orc.E1(m, uh0) + kw["D0"])
            assert abs(ro - r0) < 1e-12 * ro
            o_prev = uh0
            o_cur, rc = orc.sav_step(m, uh0, None, ro, ro, sched[0], -1.0)
            ro_prev = ro
            for i in range(1, len(sched)):
                nxt, rn = orc.sav_step(m, o_cur, o_prev, rc, ro_prev, sched[i], sched[i - 1])
                o_prev, o_cur, ro_prev, rc = o_cur, nxt, rc, rn
            assert abs(rc - rs[0]) < 1e-9 * abs(rc)
        assert rel(host(cur), o_cur) < 1e-8, scheme


def test_temporal_convergence_on_paper_data(F):
    """Fixed-step errors at T = 0.32 on the sub-critical benchmark's initial data
    (256^2) against a fine PSD reference, the comparison of Table tab:rates:
    every scheme converges at second order, PSD is the most accurate, SAV's
    errors equal IMEX's, and ETDRK2's are the largest at equal k."""
    log("temporal convergence, sub-critical 256^2")
    from paper_2006_04784_amd import sweeps
    ks = [0.01, 0.005, 0.0025, 0.00125]
    r = sweeps.temporal_convergence(ks=ks)
    rate = lambda e: [np.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]
    for sch in ("psd", "imex", "sav"):
        assert min(rate(r[sch])) > 1.75, (sch, r[sch])
    assert rate(r["etd"])[-1] > 1.5, r["etd"]
    for i in range(len(ks)):
        assert r["psd"][i] < 0.1 * r["imex"][i]
        assert abs(r["sav"][i] - r["imex"][i]) < 0.02 * r["imex"][i]
        assert r["etd"][i] > 2.0 * r["imex"][i]


@pytest.mark.parametrize("scheme", ["imex", "etd", "sav", "psd"])
def test_adaptive_device_control_matches_host_loop(F, orc, scheme):
    """fch_run's adaptive runs take their attempts under device control (the
    ensemble's batched kernels and per-member controller on a one-member view
    of the plan; SAV's r history rotates on the device; PSD solves run in
    queued rounds whose stages each run only in their phase of the attempt);
    with kernel timing on they fall back to the host loop.  Both take the
    same decisions and reach the same state (and SAV scalars, PSD iteration
    counts); the step limit and the final time are honoured exactly."""
    log("adaptive %s: device control vs host loop" % scheme)
    N, L = 256, 4 * np.pi
    plan, m = pair(F, orc, **model_kw(N, L))
    uh0 = orc.r2c(inputs.circle_bilayer(N, L, 0.1, seed=4))
    opts = F.AdaptOpts(sigma_tol=1e-5, k_max=0.05 if scheme == "psd" else float("inf"))
    res = []
    for prof in (False, True):
        plan.profile(prof)
        plan.reset_stats()
        a, b = dev(uh0), torch.zeros_like(dev(uh0))
        info = plan.run(a, b, scheme=scheme, adaptive=True, startup=True, t_end=0.05,
                        nsteps=100000, adapt=opts)
        info["launches"] = plan.stats()["launches"]
        res.append((host(a), host(b), info))
        if prof:
            plan.profile_read()
            plan.profile(False)
    (a0, b0, i0), (a1, b1, i1) = res
    log("  device: %s" % {k: i0[k] for k in ("accepted", "rejected", "psd_iters", "launches")})
    log("  host:   %s" % {k: i1[k] for k in ("accepted", "rejected", "psd_iters", "launches")})
    assert i0["accepted"] == i1["accepted"] and i0["rejected"] == i1["rejected"]
    if scheme == "psd":
        assert i0["psd_iters"] == i1["psd_iters"] and i0["fft_calls"] == i1["fft_calls"]
        # two launches per iteration plus a few per attempt: the initial
        # iterate, the F(u~) evaluation and the controller (5), iterations
        # queued after the solve stopped, a second round when an attempt
        # outruns its queued iterations; and the rounds queued after the end
        attempts = i0["accepted"] + i0["rejected"]
        assert i0["launches"] <= 2 * i0["psd_iters"] + 16 * attempts + 400
    assert abs(i0["t"] - 0.05) < 1e-15 and abs(i1["t"] - 0.05) < 1e-15
    # the error estimate is a small difference of states, so rounding differences
    # between the two kernel sets (FMA contraction) reach it at about 1e-11
    assert abs(i0["k_next"] - i1["k_next"]) <= 1e-9 * i1["k_next"]
    assert rel(a0, a1) < 1e-12 and rel(b0, b1) < 1e-12
    if scheme == "sav":
        for x, y in zip(i0["rs"], i1["rs"]):
            assert abs(x - y) <= 1e-12 * abs(y)
    # a step limit stops the run after exactly that many accepted steps
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    info = plan.run(a, b, scheme=scheme, adaptive=True, startup=True, t_end=10.0, nsteps=37,
                    adapt=opts)
    assert info["accepted"] == 37 and info["t"] < 10.0
    # a run that ends with its startup step reports that step as the next trial
    info = plan.run(a, b, scheme=scheme, adaptive=True, startup=True, t_end=1e-6, k_first=1e-6,
                    adapt=opts)
    assert info["accepted"] == 1 and info["k_next"] == 1e-6


def test_psd_iterations_match_table_tolPSD(F):
    """Adaptive BDF2-PSD on the sub-critical benchmark's initial data (256^2,
    sigma_tol 1e-5, i_tol = nu sigma_tol with nu = 1e-3 and k_max = 0.05 from
    Table tolPSD, lambda from Table SearchSize) to T = 250: the total iteration
    count lands within 15% of the 38.2 thousand the paper prints for q = 0 at
    that k_max (its row spans 34.8k-41.4k over k_max)."""
    log("psd iterations, sub-critical 256^2 to T = 250")
    from paper_2006_04784_amd import sweeps
    r = sweeps.scheme_comparison(["sub-critical"], schemes=("psd",))
    it = r["sub-critical"]["runs"]["psd"]["psd_iters"]
    assert abs(it - 38200) < 0.15 * 38200, it


def test_largest_grid_4096(F, orc):
    """N = 4096, the largest supported grid (its fused column epilogues spill
    registers): transforms, the fused IMEX chain (startup and one BDF2 step)
    and an ETDRK2 step against the oracle."""
    log("4096^2: transforms, IMEX chain, ETDRK2 step")
    N, L = 4096, 64 * np.pi
    kw = model_kw(N, L)
    plan, m = pair(F, orc, **kw)
    u0 = inputs.circle_bilayer(N, L, 0.1, seed=5)
    uh0 = orc.r2c(u0)
    uh = plan.forward(torch.from_numpy(u0).cuda())
    assert rel(host(uh), uh0) < 1e-13
    assert rel(plan.inverse(uh).cpu().numpy(), u0) < 1e-13
    ref = orc.run_fixed(m, "imex", uh0, 1e-3, 2)
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    plan.run(a, b, scheme="imex", nsteps=2, k=1e-3)
    assert rel(host(a), ref) < 1e-10
    e = plan.step_etd(dev(uh0), 1e-3)
    assert rel(host(e), orc.etd_step(m, uh0, 1e-3)) < 1e-10


def test_largest_grid_4096_sav_psd(F, orc):
    """N = 4096: the sums folded into the next kernel span the most partials
    here (N / R = 4096 row partials, N/2 + 1 = 2049 column partials), so each
    lane takes them in several rounds of preloaded loads.  A single SAV step,
    the fused SAV chain (r^{n+1} solved in every workgroup of the column pass)
    and two PSD iterations (the stopping test's ratio) against the oracle."""
    log("4096^2: SAV step, SAV chain, PSD iterations")
    N, L = 4096, 64 * np.pi
    kw = model_kw(N, L)
    plan, m = pair(F, orc, **kw)
    uh0 = orc.r2c(inputs.circle_bilayer(N, L, 0.1, seed=5))
    k = 1e-3
    r0 = float(np.sqrt(orc.E1(m, uh0) + m.D0))
    assert abs(plan.sav_r(dev(uh0)) - r0) < 1e-12 * r0
    u1, r1 = orc.sav_step(m, uh0, None, r0, r0, k, -1.0)
    u2, r2 = orc.sav_step(m, u1, uh0, r1, r0, 1.3 * k, k)
    g2, q2 = plan.step_sav(dev(u1), dev(uh0), r1, r0, 1.3 * k, k)
    assert rel(host(g2), u2) < 1e-10 and abs(q2 - r2) < 1e-12 * abs(r2)
    u3, r3 = orc.sav_step(m, u1, uh0, r1, r0, k, k)
    a, b = dev(uh0), torch.zeros_like(dev(uh0))
    info = plan.run(a, b, scheme="sav", nsteps=3, k=k)
    ref3, _ = orc.sav_step(m, u3, u1, r3, r1, k, k)
    assert rel(host(a), ref3) < 1e-10 and rel(host(b), u3) < 1e-10
    ref, it, ratio, _ = orc.psd_step(m, u1, uh0, k, k, fixed_iters=2)
    out, st = plan.step_psd(dev(u1), dev(uh0), k, k, fixed_iters=2)
    log("  SAV step %.1e, chain %.1e, PSD %.1e, ratio %.3e / %.3e"
        % (rel(host(g2), u2), rel(host(a), ref3), rel(host(out), ref), st["last_ratio"], ratio))
    assert st["iters"] == 2 and rel(host(out), ref) < 1e-10
    assert abs(st["last_ratio"] - ratio) < 1e-6 * ratio
