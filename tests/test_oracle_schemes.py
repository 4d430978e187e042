"""Pins of the oracle's time stepping:
 * BDF2 / AM3 coefficients (eqs. BDF2Coef, AM3-general, Predictor): exactness
   on polynomials and the uniform-step values printed in the paper;
 * IMEX and PSD steps in the linear regime about u = b_- (each Fourier mode
   follows a scalar three-term recurrence);
 * SAV: the identity u_SAV - u_IMEX = (xi - 1) s* q at beta = (2, 1), where the
   SAV operator L_0 equals L_IMEX (Sec. 3.5), and the modified-energy law of
   Theorem t:SAV at fixed k;
 * PSD: the converged iterate solves the fully implicit BDF2 equation;
 * second-order convergence on a manufactured solution (all three schemes);
 * mass conservation and energy decay on the 64^2 circle workload;
 * the step-size controller (Sec. 3.2, Step 4) on scripted error values;
 * the lambda(q, k) table (Table SearchSize)."""
import os

import numpy as np
import pytest

from paper_2006_04784_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_bdf2_coefficients_exact_for_quadratics(orc):
    rng = np.random.default_rng(0)
    for _ in range(20):
        k1, k0 = rng.uniform(1e-3, 1.0, size=2)
        a, b, c = orc.bdf2_coef(k1, k0)
        assert abs(a + b + c) < 1e-12 * abs(a)
        t1, t0, tm = 0.3 + k0 + k1, 0.3 + k0, 0.3
        for (p0, p1, p2) in [(1.0, 0, 0), (0.2, 1.0, 0), (0.1, -0.5, 2.0)]:
            u = lambda t: p0 + p1 * t + p2 * t * t
            du = p1 + 2 * p2 * t1
            assert abs(a * u(t1) + b * u(t0) + c * u(tm) - du) < 1e-9 * (1 + abs(du)) * a * k1


def test_uniform_step_golden(orc):
    rows = {}
    for line in open(os.path.join(GOLDEN, "uniform_step_coefficients.txt")):
        if line.strip() and not line.startswith("#"):
            name, *vals = line.split()
            rows[name] = np.array(vals, float)
    k = 0.37
    a, b, c = orc.bdf2_coef(k, k)
    assert np.allclose(np.array([a, b, c]) * 2 * k, rows["bdf2"], rtol=0, atol=1e-14)
    w = np.array(orc.am3_weights(k, k)) / k
    assert np.allclose(w, rows["am3"], rtol=0, atol=1e-15)
    # startup step (k_n <= 0): first-order BDF
    a, b, c = orc.bdf2_coef(k, -1.0)
    assert (a, b, c) == (1 / k, -1 / k, 0.0)


def test_am3_exact_for_quadratic_F(orc):
    rng = np.random.default_rng(1)
    for _ in range(20):
        k1, k0 = rng.uniform(1e-3, 1.0, size=2)
        w1, w2, w3 = orc.am3_weights(k1, k0)
        assert abs(w1 + w2 + w3 - k1) < 1e-14
        tm, t0 = 0.1, 0.1 + k0
        t1 = t0 + k1
        c = rng.standard_normal(3)
        F = lambda t: c[0] + c[1] * t + c[2] * t * t
        Fint = lambda t: c[0] * t + c[1] * t * t / 2 + c[2] * t**3 / 3
        assert abs(w1 * F(t1) + w2 * F(t0) + w3 * F(tm) - (Fint(t1) - Fint(t0))) < 1e-13


def _linear_setup(orc, N=32, L=2 * np.pi, eps=0.2, q=0.0):
    m = orc.Model(N=N, L=L, eps=eps, eta1=1.45, eta2=2.0, q=q)
    X, Y = inputs.grid(N, L)
    modes = [(1, 2), (3, 0), (5, 4)]
    return m, X, Y, modes


@pytest.mark.parametrize("scheme,beta", [("imex", (2.0, 1.0)), ("imex", (1.0, 2.0)),
                                         ("imex", (2.75, 0.25)), ("psd", (2.0, 1.0))])
def test_linear_regime_recurrence(orc, scheme, beta):
    m, X, Y, modes = _linear_setup(orc)
    m.beta1, m.beta2 = beta
    eps, al = m.eps, orc.alpha_m(m)
    eta1, eta2 = m.eta1 * eps, m.eta2 * eps
    delta = 1e-7
    k1, k0 = 0.013, 0.01
    a, b, c = orc.bdf2_coef(k1, k0)
    g = k1 / k0
    un = -1.0 + 0 * X
    um = -1.0 + 0 * X
    amp_n = [1.0, -0.5, 0.7]
    amp_m = [0.8, -0.3, 0.9]
    for (mx, my), an, am in zip(modes, amp_n, amp_m):
        ph = 2 * np.pi * (mx * X + my * Y) / m.L
        un = un + delta * an * np.cos(ph)
        um = um + delta * am * np.cos(ph)
    uhn, uhm = orc.r2c(un), orc.r2c(um)
    if scheme == "imex":
        out = orc.imex_step(m, uhn, uhm, k1, k0)
    else:
        out, it, _, rc = orc.psd_step(m, uhn, uhm, k1, k0, tol=1e-13, lam=1.0)
        assert rc == 0
    N = m.N
    for (mx, my), an, am in zip(modes, amp_n, amp_m):
        k2 = (2 * np.pi / m.L) ** 2 * (mx * mx + my * my)
        Lk = (eps * eps * k2 + al) ** 2
        vs = an + g * (an - am)
        if scheme == "imex":
            # linearized mu about b_-: [(eps^2 k2 + alpha)^2 - eps^2 eta1 k2 - eta2 alpha] v,
            # split as L_0(beta) v + the explicit remainder
            L0 = (eps * eps * k2) ** 2 + beta[0] * al * eps * eps * k2 + beta[1] * al * al
            expl = Lk - eps * eps * eta1 * k2 - eta2 * al - L0
            pred = (-b * an - c * am - k2 * expl * vs) / (a + k2 * L0)
        else:
            sigma = Lk - eps * eps * eta1 * k2 - eta2 * al
            pred = (-b * an - c * am) / (a + k2 * sigma)
        got = 2 * out[my % N, mx].real / (N * N) / delta
        assert abs(got - pred) < 1e-5 * abs(pred), (mx, my, got, pred)
    # zero mode (mass) untouched
    assert abs(out[0, 0] - uhn[0, 0]) < 1e-12 * abs(uhn[0, 0])


def _c1(orc):
    kw, u0 = inputs.workload("c1")
    m = orc.Model(**kw, zeta=1.1, D0=163.0)
    return m, orc.r2c(u0)


@pytest.mark.parametrize("beta", [(2.0, 1.0), (1.0, 2.0), (0.5, 2.5)])
def test_sav_minus_imex_identity(orc, beta):
    """With the same stabilized L_0(beta) (eq. e:SAV-L0) in both schemes, SAV with
    r^{n+1} = s* is the IMEX step, so u_SAV - u_IMEX = (xi - 1) s* q."""
    m, uh0 = _c1(orc)
    m.beta1, m.beta2 = beta
    k = 1e-3
    u1 = orc.imex_step(m, uh0, None, k, -1.0)
    r0 = float(np.sqrt(orc.E1(m, uh0) + m.D0))
    # a nontrivial r^n so that xi = r^{n+1}/s* differs from 1
    rn, rm = 1.01 * r0, r0
    ui = orc.imex_step(m, u1, uh0, 1.3 * k, k)
    us, r1, s, qh = orc.sav_step(m, u1, uh0, rn, rm, 1.3 * k, k, want_q=True)
    xi = r1 / s
    lhs = us - ui
    rhs = (xi - 1.0) * s * qh
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(ui) + 1e-12 * np.linalg.norm(rhs)
    assert abs(xi - 1.0) > 1e-4          # the identity was exercised


def test_sav_modified_energy_decays(orc):
    """Theorem t:SAV: E_aux(u^{n+1}, u^n, r^{n+1}, r^n) <= E_aux(u^n, u^{n-1}, r^n, r^{n-1}) at fixed k."""
    m, uh0 = _c1(orc)
    k = 2e-3
    r0 = float(np.sqrt(orc.E1(m, uh0) + m.D0))
    u1, r1 = orc.sav_step(m, uh0, None, r0, r0, k, -1.0)
    prev = orc.E_aux(m, u1, uh0, r1, r0)
    un, um, rn, rm = u1, uh0, r1, r0
    for _ in range(25):
        new, rnew = orc.sav_step(m, un, um, rn, rm, k, k)
        um, un, rm, rn = un, new, rn, rnew
        cur = orc.E_aux(m, un, um, rn, rm)
        assert cur <= prev + 1e-12 * abs(prev)
        prev = cur


def test_psd_converged_solves_bdf2(orc):
    m, uh0 = _c1(orc)
    k = 1e-3
    u1 = orc.imex_step(m, uh0, None, k, -1.0)
    tol = 1e-10
    u2, it, ratio, rc = orc.psd_step(m, u1, uh0, k, k, tol=tol)
    assert rc == 0 and ratio < tol and it > 1
    a, b, c = orc.bdf2_coef(k, k)
    N, L, eps = m.N, m.L, m.eps
    al = orc.alpha_m(m)
    kx = 2 * np.pi * np.arange(N // 2 + 1) / L
    ky = 2 * np.pi * np.fft.fftfreq(N, d=1.0 / N) / L
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    res = a * u2 + b * u1 + c * uh0 - orc.F(m, u2)
    k2s = np.where(k2 == 0, 1.0, k2)
    pre = res / (k2s * ((eps * eps * k2 + al) ** 2 + a / k2s))
    pre[0, 0] = 0.0
    assert np.linalg.norm(pre) / np.linalg.norm(u2) < 10 * tol
    assert abs(res[0, 0]) < 1e-9 * abs(u2[0, 0]) * a


def test_psd_fixed_iterations_and_noconv(orc):
    m, uh0 = _c1(orc)
    k = 1e-3
    u1 = orc.imex_step(m, uh0, None, k, -1.0)
    _, it, _, rc = orc.psd_step(m, u1, uh0, k, k, fixed_iters=3)
    assert it == 3 and rc == 0
    _, it, _, rc = orc.psd_step(m, u1, uh0, k, k, tol=1e-30, max_iter=4)
    assert it == 4 and rc == 1


# ---- manufactured solution -------------------------------------------------
def _manufactured(orc, scheme, nsteps, T=0.5):
    N, L = 32, 2 * np.pi
    m = orc.Model(N=N, L=L, eps=0.1, eta1=1.45, eta2=2.0, zeta=1.1, D0=1000.0)
    X, Y = inputs.grid(N, L)
    # stays near b_- = -1, the state the IMEX split is built to stabilize
    # (Sec. 3.4); far from it the explicit part of the split is not stable
    ue = lambda t: -0.95 + 0.1 * np.cos(t) * np.cos(X) * np.cos(Y) + 0.05 * np.sin(2 * t) * np.sin(2 * X)
    ut = lambda t: -0.1 * np.sin(t) * np.cos(X) * np.cos(Y) + 0.1 * np.cos(2 * t) * np.sin(2 * X)
    forcing = lambda t: orc.r2c(ut(t)) - orc.F(m, orc.r2c(ue(t)))
    k = T / nsteps
    um, un = orc.r2c(ue(0.0)), orc.r2c(ue(k))
    rm = float(np.sqrt(orc.E1(m, um) + m.D0))
    rn = float(np.sqrt(orc.E1(m, un) + m.D0))
    for n in range(1, nsteps):
        f = forcing((n + 1) * k)
        if scheme == "imex":
            new = orc.imex_step(m, un, um, k, k, fh=f)
        elif scheme == "sav":
            new, rnew = orc.sav_step(m, un, um, rn, rm, k, k, fh=f)
            rm, rn = rn, rnew
        else:
            new, it, ratio, rc = orc.psd_step(m, un, um, k, k, fh=f, tol=1e-13, lam=1.0,
                                              max_iter=5000)
            assert rc == 0
        um, un = un, new
    err = np.linalg.norm(orc.c2r(un) - ue(T)) / np.linalg.norm(ue(T))
    return err


@pytest.mark.parametrize("scheme", ["imex", "sav", "psd"])
def test_manufactured_second_order(orc, scheme):
    ms = [32, 64, 128] if scheme != "psd" else [16, 32, 64]
    errs = [_manufactured(orc, scheme, n) for n in ms]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) >= 1.9, (errs, rates)


def test_c1_mass_and_energy(orc):
    m, uh0 = _c1(orc)
    un, states = orc.run_fixed(m, "imex", uh0, 1e-3, 60, record=True)
    m0 = orc.mass(m, uh0)
    E = [orc.energy(m, s) for s in states]
    for s in states[1:]:
        assert abs(s[0, 0] - uh0[0, 0]) <= 1e-13 * abs(uh0[0, 0])
    assert abs(orc.mass(m, un) - m0) < 1e-12 * m0
    assert all(E[i + 1] <= E[i] for i in range(len(E) - 1))


def test_adapt_controller_scripted(orc):
    cap = 1 + np.sqrt(2)
    sig, kmin, kmax = 1e-5, 1e-9, np.inf
    acc, kn = orc.adapt_decide(sig / 8, 1e-3, sig, kmin, kmax)
    assert acc and abs(kn - 0.9 * 2 * 1e-3) < 1e-15
    acc, kn = orc.adapt_decide(sig / 1000, 1e-3, sig, kmin, kmax)
    assert acc and abs(kn - cap * 1e-3) < 1e-15
    acc, kn = orc.adapt_decide(8 * sig, 1e-3, sig, kmin, kmax)
    assert not acc and abs(kn - 0.45e-3) < 1e-15
    acc, kn = orc.adapt_decide(1e6 * sig, kmin, sig, kmin, kmax)
    assert acc and kn == kmin
    acc, kn = orc.adapt_decide(0.0, 1e-3, sig, kmin, 0.05)
    assert acc and kn == pytest.approx(cap * 1e-3)
    acc, kn = orc.adapt_decide(sig / 1000, 0.04, sig, kmin, 0.05)
    assert acc and kn == 0.05
    acc, kn = orc.adapt_decide(sig / 1000, 1e-3, sig, kmin, kmax, cap=0.0)
    assert acc and kn == pytest.approx(0.9 * 10 * 1e-3)


def test_am3_error_zero_and_one(orc):
    m, uh0 = _c1(orc)
    rng = np.random.default_rng(5)
    shp = uh0.shape
    Fs = [orc.r2c(rng.standard_normal((m.N, m.N))) for _ in range(3)]
    k1, k0 = 2e-3, 1e-3
    w1, w2, w3 = orc.am3_weights(k1, k0)
    up = uh0 + w1 * Fs[0] + w2 * Fs[1] + w3 * Fs[2]
    assert orc.am3_error(m, up, uh0, Fs[0], Fs[1], Fs[2], k1, k0) < 1e-14
    assert abs(orc.am3_error(m, 2 * up, uh0, Fs[0], Fs[1], Fs[2], k1, k0) - 1.0) < 1e-13
    assert shp == up.shape


def test_lambda_table(orc):
    lines = [l.split() for l in open(os.path.join(GOLDEN, "lambda_search_size.txt"))
             if l.strip() and not l.startswith("#")]
    ks = np.array(lines[0][1:], float)
    for row in lines[1:]:
        q, lam = float(row[0]), np.array(row[1:], float)
        for kk, ll in zip(ks, lam):
            assert abs(orc.lambda_table(q, kk) - ll) < 1e-14
        mid = 0.5 * (ks[3] + ks[4])
        assert abs(orc.lambda_table(q, mid) - 0.5 * (lam[3] + lam[4])) < 1e-12
        assert orc.lambda_table(q, 1e-9) == lam[0] and orc.lambda_table(q, 0.5) == lam[-1]
    assert orc.lambda_table(0.3, 1e-3) < 0
