"""Seeded synthetic initial states for the FCH benchmarks.

This module only draws and shapes input fields (numpy PCG64 streams); it holds
none of the scheme's arithmetic.  Both the GPU path and the CPU oracle are fed
from it, so a test can hand identical inputs to each side.

Bilayer dressing of a closed curve: with s the signed radial distance to the
curve and half-width R = 1.4725*eps (the paper's strip half-width 0.14725 at
eps = 0.1, Sec. 2.3), the indicator is smoothed to
    phi(s) = (tanh((s + R)/eps) - tanh((s - R)/eps)) / 2
and u = u_bg + (b_+ - u_bg) * max_j phi_j.  Distances use periodic minimum
images on [0, L)^2.  Grid point (i, j) sits at (x, y) = (j h, i h).
"""
from __future__ import annotations

import numpy as np

R_OVER_EPS = 1.4725


def grid(N: int, L: float):
    h = L / N
    x = np.arange(N) * h
    X, Y = np.meshgrid(x, x, indexing="xy")   # X[i, j] = j h, Y[i, j] = i h
    return X, Y


def _min_image(d, L):
    return d - L * np.round(d / L)


def bilayer_phi(s, eps):
    R = R_OVER_EPS * eps
    return 0.5 * (np.tanh((s + R) / eps) - np.tanh((s - R) / eps))


def circle_bilayer(N: int, L: float, eps: float, radius_frac: float = 0.3,
                   u_bg: float = -0.99, noise: float = 1e-3, seed: int = 0,
                   b_plus: float = 1.0):
    """One circular bilayer of radius radius_frac*L centred in the box on a
    constant background, plus i.i.d. N(0, noise^2) per grid point."""
    X, Y = grid(N, L)
    dx = _min_image(X - L / 2, L)
    dy = _min_image(Y - L / 2, L)
    s = np.hypot(dx, dy) - radius_frac * L
    u = u_bg + (b_plus - u_bg) * bilayer_phi(s, eps)
    rng = np.random.default_rng(seed)
    if noise > 0:
        u = u + rng.normal(0.0, noise, size=(N, N))
    return u


def perturbed_circles(N: int, L: float, eps: float, count: int, seed: int = 0,
                      r_range=(0.5, 2.0), amp_max: float = 0.05,
                      mass_excess=(0.01, 0.05), u_bg: float | None = None,
                      noise: float = 1e-4, min_gap_eps: float = 10.0,
                      b_plus: float = 1.0, max_tries: int = 20000):
    """`count` closed bilayers rho(theta) = r [1 + sum_{m=2..4} a_m cos(m(theta - phi_m))]
    at uniformly drawn centres (placements closer than min_gap_eps*eps between
    bands are redrawn), on a background -1 + delta with delta ~ U(mass_excess)
    unless u_bg is given, plus N(0, noise^2)."""
    rng = np.random.default_rng(seed)
    X, Y = grid(N, L)
    curves = []
    tries = 0
    while len(curves) < count and tries < max_tries:
        tries += 1
        r = rng.uniform(*r_range)
        amps = rng.uniform(0.0, amp_max, size=3)
        phs = rng.uniform(0.0, 2 * np.pi, size=3)
        c = rng.uniform(0.0, L, size=2)
        rmax = r * (1.0 + amps.sum())
        ok = True
        for (c2, r2max, *_rest) in curves:
            d = np.hypot(*_min_image(np.asarray(c) - c2, L))
            if d < rmax + r2max + min_gap_eps * eps:
                ok = False
                break
        if ok and 2 * rmax + min_gap_eps * eps < L:
            curves.append((np.asarray(c), rmax, r, amps, phs))
    if len(curves) < count:
        raise ValueError("could not place %d curves" % count)
    phi = np.zeros((N, N))
    for (c, _rmax, r, amps, phs) in curves:
        dx = _min_image(X - c[0], L)
        dy = _min_image(Y - c[1], L)
        th = np.arctan2(dy, dx)
        rho = r * (1.0 + sum(amps[m] * np.cos((m + 2) * (th - phs[m])) for m in range(3)))
        s = np.hypot(dx, dy) - rho
        phi = np.maximum(phi, bilayer_phi(s, eps))
    if u_bg is None:
        u_bg = -1.0 + rng.uniform(*mass_excess)
    u = u_bg + (b_plus - u_bg) * phi
    if noise > 0:
        u = u + rng.normal(0.0, noise, size=(N, N))
    return u


def gaussian_random_field(N: int, L: float, corr_len: float, std: float, seed: int = 0):
    """White noise filtered by exp(-|k|^2 l^2 / 4) (covariance ~ exp(-r^2/(2 l^2))),
    mean removed and scaled to the given standard deviation."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((N, N))
    k1 = 2 * np.pi * np.fft.fftfreq(N, d=L / N)
    k2 = k1[:, None] ** 2 + k1[None, :] ** 2
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * np.exp(-k2 * corr_len ** 2 / 4.0)))
    f -= f.mean()
    return f * (std / f.std())


def white_noise(N: int, seed: int = 0, scale: float = 1.0):
    """Seeded N(0, scale^2) field, for transform tests."""
    return np.random.default_rng(seed).normal(0.0, scale, size=(N, N))


# ---- named workloads -------------------------------------------------------
def workload(name: str, seed: int = 0):
    """(model keyword arguments, physical initial state) of a named workload.

    c1: 64^2 on [0, 4 pi]^2, eps 0.1, one circle of radius 0.3 L, background -0.99
    c2: 512^2 on [0, 8 pi]^2, eps 0.05, six perturbed circles, raised background
    c3: 2048^2 on [0, 16 pi]^2, eps 0.05, forty perturbed circles + GRF (l = 4 eps)
    c5: 256^2 on [0, 4 pi]^2, eps 0.05, three perturbed circles
    m1: 1024^2 on [0, 16 pi]^2, eps 0.1, one circle of radius 0.3 L (c1 scaled)
    """
    if name == "c1":
        kw = dict(N=64, L=4 * np.pi, eps=0.1, eta1=1.45, eta2=2.0)
        return kw, circle_bilayer(64, kw["L"], 0.1, seed=seed)
    if name == "m1":
        kw = dict(N=1024, L=16 * np.pi, eps=0.1, eta1=1.45, eta2=2.0)
        return kw, circle_bilayer(1024, kw["L"], 0.1, seed=seed)
    if name == "c2":
        kw = dict(N=512, L=8 * np.pi, eps=0.05, eta1=1.45, eta2=2.0)
        return kw, perturbed_circles(512, kw["L"], 0.05, 6, seed=seed)
    if name == "c3":
        kw = dict(N=2048, L=16 * np.pi, eps=0.05, eta1=1.45, eta2=2.0)
        u = perturbed_circles(2048, kw["L"], 0.05, 40, seed=seed, u_bg=-0.99, noise=0.0)
        u = u + gaussian_random_field(2048, kw["L"], 4 * 0.05, 1e-3, seed=seed + 1)
        return kw, u
    if name == "c5":
        kw = dict(N=256, L=4 * np.pi, eps=0.05, eta1=1.45, eta2=2.0)
        return kw, perturbed_circles(256, kw["L"], 0.05, 3, seed=seed, r_range=(0.5, 1.5))
    raise KeyError(name)
