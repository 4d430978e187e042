"""Pins of the oracle's model pieces: the regularized well W_q (eq. e:Wq-def)
against closed forms, finite differences and the alpha_m column of Table
t:Benchmark; the chemical potential (eq. FCH) against an analytic evaluation
with exact derivatives; energy, E_1 and V against their variational
derivatives; mass and the L2 inner product against closed forms."""
import os

import numpy as np
import pytest

from paper_2006_04784_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def model(orc, **kw):
    base = dict(N=32, L=2 * np.pi, eps=0.1, eta1=1.45, eta2=2.0)
    base.update(kw)
    return orc.Model(**base)


def test_well_q0_closed_forms(orc):
    m = model(orc, q=0.0)
    u = np.linspace(-2.0, 2.0, 401)
    W, W1, W2 = orc.well(m, u)
    assert np.max(np.abs(W - (0.25 * u**4 + 0.05 * u**3 - 0.5 * u**2 - 0.15 * u + 0.15))) < 1e-14
    assert np.max(np.abs(W1 - (u * u - 1.0) * (u + 0.15))) < 1e-14
    assert np.max(np.abs(W2 - (3 * u * u + 0.3 * u - 1.0))) < 1e-14
    # roots of W' for q = 0
    _, r1, _ = orc.well(m, np.array([-1.0, -0.15, 1.0]))
    assert np.max(np.abs(r1)) < 1e-15


def test_alpha_m_table1(orc):
    rows = np.loadtxt(os.path.join(GOLDEN, "table1_alpha_m.txt"))
    for q, eps, alpha in rows:
        m = model(orc, q=q, eps=eps)
        assert abs(orc.alpha_m(m) - alpha) < 1e-13


@pytest.mark.parametrize("q", [0.0, 0.2, 0.5])
def test_well_double_zero_at_bminus(orc, q):
    m = model(orc, q=q)
    W, W1, _ = orc.well(m, np.array([-1.0]))
    assert abs(W[0]) < 1e-15 and abs(W1[0]) < 1e-15


@pytest.mark.parametrize("q", [0.2, 0.5])
def test_well_derivatives_finite_difference(orc, q):
    m = model(orc, q=q)
    u = np.linspace(-1.6, 1.4, 97)
    h = 1e-5
    W, W1, W2 = orc.well(m, u)
    Wp, W1p, _ = orc.well(m, u + h)
    Wm, W1m, _ = orc.well(m, u - h)
    assert np.max(np.abs((Wp - Wm) / (2 * h) - W1)) < 1e-8 * max(1, np.max(np.abs(W1)))
    assert np.max(np.abs((W1p - W1m) / (2 * h) - W2)) < 1e-6 * max(1, np.max(np.abs(W2)))


def _analytic_mu(X, Y, c0, A, B, Cc, eps, eta1, eta2):
    """mu of eq. FCH for u = c0 + A cos x + B sin 2y + C cos(x+y) with q = 0,
    using exact derivatives and Lap W'(u) = W'''|grad u|^2 + W'' Lap u."""
    u = c0 + A * np.cos(X) + B * np.sin(2 * Y) + Cc * np.cos(X + Y)
    ux = -A * np.sin(X) - Cc * np.sin(X + Y)
    uy = 2 * B * np.cos(2 * Y) - Cc * np.sin(X + Y)
    lap = -A * np.cos(X) - 4 * B * np.sin(2 * Y) - 2 * Cc * np.cos(X + Y)
    lap2 = A * np.cos(X) + 16 * B * np.sin(2 * Y) + 4 * Cc * np.cos(X + Y)
    W1 = (u * u - 1) * (u + 0.15)
    W2 = 3 * u * u + 0.3 * u - 1
    W3 = 6 * u + 0.3
    lapW1 = W3 * (ux * ux + uy * uy) + W2 * lap
    e2 = eps * eps
    omega = e2 * lap - W1
    lap_omega = e2 * lap2 - lapW1
    return u, e2 * lap_omega - W2 * omega + e2 * eta1 * lap - eta2 * W1


def test_mu_against_analytic(orc):
    N, L, eps = 32, 2 * np.pi, 0.3
    m = model(orc, N=N, L=L, eps=eps, eta1=1.45, eta2=2.0, p=1)
    X, Y = inputs.grid(N, L)
    u, mu_exact = _analytic_mu(X, Y, -0.4, 0.3, 0.2, 0.25, eps, 1.45 * eps, 2.0 * eps)
    uh = orc.r2c(u)
    mu = orc.c2r(orc.mu(m, uh))
    assert np.linalg.norm(mu - mu_exact) / np.linalg.norm(mu_exact) < 1e-12
    # F = Lap mu, with the (separately pinned) spectral Laplacian
    F = orc.c2r(orc.F(m, uh))
    # (the Laplacian amplifies rounding in the high modes by up to |k|^2 ~ 500)
    assert np.linalg.norm(F - orc.laplacian(m, mu_exact)) / np.linalg.norm(F) < 1e-10


def _field(orc, N, L, seed):
    X, Y = inputs.grid(N, L)
    rng = np.random.default_rng(seed)
    u = -0.3 + 0.0 * X
    for _ in range(4):
        a, b = rng.integers(-3, 4, size=2)
        u = u + 0.2 * rng.uniform(-1, 1) * np.cos(2 * np.pi * (a * X + b * Y) / L + rng.uniform(0, 6))
    return u


@pytest.mark.parametrize("q", [0.0, 0.2])
def test_energy_gradient_is_mu(orc, q):
    """d/ds E(u + s v) at s = 0 equals (mu(u), v): the discrete energy and the
    chemical potential are consistent (eq. Functional vs eq. FCH)."""
    N, L = 32, 2 * np.pi
    m = model(orc, N=N, L=L, eps=0.3, q=q)
    u = _field(orc, N, L, 1)
    v = _field(orc, N, L, 2) + 0.3
    uh, vh = orc.r2c(u), orc.r2c(v)
    s = 1e-5
    dE = (orc.energy(m, uh + s * vh) - orc.energy(m, uh - s * vh)) / (2 * s)
    pred = orc.inner(m, orc.mu(m, uh), vh)
    assert abs(dE - pred) < 1e-7 * max(1.0, abs(pred))


@pytest.mark.parametrize("q", [0.0, 0.5])
def test_E1_gradient_is_V_and_split(orc, q):
    """d/ds E_1(u + s v) = (V(u), v) (eq. e:G-def), and L_SAV u + V = mu (eq. 4.2-4.3)."""
    N, L, eps = 32, 2 * np.pi, 0.3
    m = model(orc, N=N, L=L, eps=eps, q=q, zeta=1.1)
    u = _field(orc, N, L, 3)
    v = _field(orc, N, L, 4)
    uh, vh = orc.r2c(u), orc.r2c(v)
    s = 1e-5
    dE = (orc.E1(m, uh + s * vh) - orc.E1(m, uh - s * vh)) / (2 * s)
    pred = orc.inner(m, orc.V(m, uh), vh)
    assert abs(dE - pred) < 1e-7 * max(1.0, abs(pred))
    # L_SAV u = eps^4 Lap^2 u + eps^2 (eta1 + 2 zeta) Lap u, eta1 effective
    lap = orc.laplacian(m, u)
    lsav = eps**4 * orc.laplacian(m, lap) + eps**2 * (1.45 * eps + 2 * 1.1) * lap
    total = lsav + orc.c2r(orc.V(m, uh))
    mu = orc.c2r(orc.mu(m, uh))
    assert np.linalg.norm(total - mu) / np.linalg.norm(mu) < 1e-12


def test_mass_and_inner_closed_forms(orc):
    N, L = 32, 4 * np.pi
    m = model(orc, N=N, L=L)
    X, Y = inputs.grid(N, L)
    u = -0.7 + 0.3 * np.cos(2 * np.pi * X / L) + 0.1 * np.sin(4 * np.pi * Y / L)
    uh = orc.r2c(u)
    assert abs(orc.mass(m, uh) - 0.5 * L * L * 0.3) < 1e-12
    c = np.cos(2 * np.pi * X / L)
    assert abs(orc.inner(m, orc.r2c(c), orc.r2c(c)) - L * L / 2) < 1e-12
