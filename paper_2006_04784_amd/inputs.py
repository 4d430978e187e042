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


# ---- the paper's benchmark initial data (Sec. 2.3, eq. dcoef, Table t:Benchmark) ----
PAPER_L = 4 * np.pi          # Omega = [0, 4 pi]^2
PAPER_N0 = 256               # mesh of the filtered strip
PAPER_R = 0.14725            # strip half-width
PAPER_LAMBDA0 = 7.0269e-3    # filter exponent
PAPER_ALPHA0 = 1.7           # alpha_m(0) = W_0''(b_-), printed in Table t:Benchmark
# Table t:Benchmark: q, eta_1/eps, eta_2/eps, d, N (eps = 0.1, gamma = 0.3) and the
# printed initial mass
PAPER_BENCHMARKS = {
    "sub-critical": dict(q=0.0, eta1=1.45, eta2=3.0, d=0.2, N=256, mass=6.11),
    "critical": dict(q=0.0, eta1=1.45, eta2=1.5, d=0.75, N=256, mass=7.61),
    "super-critical": dict(q=0.0, eta1=1.45, eta2=3.0, d=0.5, N=256, mass=6.93),
    "foot-1": dict(q=0.2, eta1=1.45, eta2=3.0, d=0.2, N=256, mass=6.11),
    "foot-2": dict(q=0.5, eta1=1.45, eta2=3.0, d=0.2, N=512, mass=6.11),
}


def paper_curve(theta, eps: float = 0.1, L: float = PAPER_L):
    """The curve Gamma in polar form about the box centre:
    rho(theta) = 3 - (eps/2) cos(6 (theta - pi/11)) - eps^2 cos(theta - 3 pi/11)."""
    rho = 3.0 - 0.5 * eps * np.cos(6.0 * (theta - np.pi / 11)) - eps * eps * np.cos(theta - 3 * np.pi / 11)
    return rho * np.cos(theta) + L / 2, rho * np.sin(theta) + L / 2


def _curve_distance(px, py, eps, L, samples=20000):
    """Distance from the points (px, py) to Gamma, taken to a closed polyline
    through `samples` points of Gamma and searched near each point's polar
    angle (Gamma is star-shaped about the box centre; the points lie within
    0.5 of radius 3)."""
    th = 2 * np.pi * np.arange(samples) / samples
    cx, cy = paper_curve(th, eps, L)
    ang = np.mod(np.arctan2(py - L / 2, px - L / 2), 2 * np.pi)
    centre = np.rint(ang / (2 * np.pi) * samples).astype(np.int64)
    best = np.full(px.shape, np.inf)
    win = samples // 200  # +-0.03 rad, several times the largest angular offset of the foot point
    for off in range(-win, win):
        i0 = np.mod(centre + off, samples)
        i1 = np.mod(i0 + 1, samples)
        ax, ay = cx[i0], cy[i0]
        bx, by = cx[i1] - ax, cy[i1] - ay
        t = np.clip(((px - ax) * bx + (py - ay) * by) / (bx * bx + by * by), 0.0, 1.0)
        best = np.minimum(best, np.hypot(px - ax - t * bx, py - ay - t * by))
    return best


def paper_strip_indicator(N0: int = PAPER_N0, eps: float = 0.1, R: float = PAPER_R,
                          L: float = PAPER_L, sub: int = 8):
    """phi_Gamma on the N0 x N0 mesh: +1 inside the strip Gamma_R between the
    offset curves Gamma_+- (the points within distance R of Gamma, R being far
    below Gamma's smallest radius of curvature), -1 outside, each mesh value
    being the average of the indicator over its cell (sub x sub points; only
    cells the strip's edge crosses need more than their centre).  sub = 1
    samples the indicator at the mesh points instead."""
    X, Y = grid(N0, L)
    h = L / N0
    phi = -np.ones((N0, N0))
    r = np.hypot(X - L / 2, Y - L / 2)
    ci, cj = np.nonzero(np.abs(r - 3.0) < 0.45)
    d = _curve_distance(X[ci, cj], Y[ci, cj], eps, L)
    if sub == 1:
        phi[ci[d < R], cj[d < R]] = 1.0
        return phi
    inner = d < R - h
    phi[ci[inner], cj[inner]] = 1.0
    edge = np.abs(d - R) <= h
    ei, ej = ci[edge], cj[edge]
    o = (np.arange(sub) + 0.5) / sub - 0.5
    ox, oy = np.meshgrid(o * h, o * h, indexing="xy")
    px = (X[ei, ej][:, None] + ox.ravel()[None, :]).ravel()
    py = (Y[ei, ej][:, None] + oy.ravel()[None, :]).ravel()
    inside = (_curve_distance(px, py, eps, L) < R).reshape(len(ei), sub * sub)
    phi[ei, ej] = 2.0 * inside.mean(axis=1) - 1.0
    return phi


def paper_initial_data(name: str, N: int = None, eps: float = 0.1, physical_k: bool = False,
                       d: float = None, sampling: str = "cell", n0: int = PAPER_N0):
    """u^0_N = phi_256 + eps d / alpha_m(0)^2 (eq. dcoef) for a benchmark of
    Table t:Benchmark.  phi_256 = F[phi_Gamma]: the DFT of the strip indicator
    on the 256 mesh times exp(-lambda0 (k1^2 + k2^2)), summed as a
    trigonometric polynomial and evaluated on the N x N grid (N >= 256).  The
    filter takes the integer mode indices k1, k2 literally; physical_k uses the
    wavenumbers 2 pi k / L instead.  d overrides the benchmark's background
    parameter.  Readings of the indicator's "interpolation" to the mesh:
    sampling = "cell" (cell averages) or "point" (values at the mesh points);
    n0: the mesh of the indicator and its DFT (256 in the text; 512 resolves
    the strip's edge better; the filter leaves no weight beyond |k| = 128).
    Returns (model keyword arguments, u0)."""
    b = PAPER_BENCHMARKS[name]
    d = b["d"] if d is None else d
    N = N or b["N"]
    N0 = n0
    if sampling not in ("cell", "point"):
        raise ValueError(sampling)
    if N < PAPER_N0 or N % PAPER_N0 or N0 % PAPER_N0:
        raise ValueError("N and n0 must be multiples of %d" % PAPER_N0)
    phi = paper_strip_indicator(N0, eps, sub=8 if sampling == "cell" else 1)
    ph = np.fft.fft2(phi)
    k = np.fft.fftfreq(N0, d=1.0 / N0)           # integer indices -N0/2 .. N0/2-1
    if physical_k:
        k = k * 2 * np.pi / PAPER_L
    ph *= np.exp(-PAPER_LAMBDA0 * (k[:, None] ** 2 + k[None, :] ** 2))
    # carry the modes |k| < M/2 over to the N grid (M = min(N, N0)); the
    # Nyquist row and column (+-M/2) split evenly when padding, and are
    # dropped when truncating (their weight, exp(-lambda0 M^2/4) < 1e-49)
    M = min(N, N0)
    big = np.zeros((N, N), complex)
    h = M // 2
    idx = np.concatenate([np.arange(h), np.arange(N - h, N)])
    src = np.concatenate([np.arange(h), np.arange(N0 - h, N0)])
    big[np.ix_(idx, idx)] = ph[np.ix_(src, src)]
    if N > N0:
        ny = big[N - h, :].copy()
        big[N - h, :] = 0.5 * ny
        big[h, :] = 0.5 * ny
        nx = big[:, N - h].copy()
        big[:, N - h] = 0.5 * nx
        big[:, h] = 0.5 * nx
    elif N < N0:
        big[N - h, :] = 0.0
        big[:, N - h] = 0.0
    phiN = np.real(np.fft.ifft2(big)) * (N / N0) ** 2
    u0 = phiN + eps * d / PAPER_ALPHA0 ** 2
    kw = dict(N=N, L=PAPER_L, eps=eps, eta1=b["eta1"], eta2=b["eta2"], q=b["q"])
    return kw, u0


# ---- named workloads -------------------------------------------------------
def c4_members(count: int = 64, seed: int = 2024):
    """Model keyword arguments of the mixed-size ensemble's members: N drawn
    from {128, 256, 512, 1024}, L = N 4 pi / 256 (h/eps = 0.49), eps 0.1,
    eta1 ~ U[1.2, 1.6], eta2 ~ U[1.5, 2.5] (times eps^p)."""
    rng = np.random.default_rng(seed)
    mem = []
    for _ in range(count):
        Ni = int(rng.choice([128, 256, 512, 1024]))
        Li = Ni * 4 * np.pi / 256
        mem.append(dict(N=Ni, L=Li, eps=0.1, eta1=float(rng.uniform(1.2, 1.6)),
                        eta2=float(rng.uniform(1.5, 2.5))))
    return mem


def c4_initial(member: dict, index: int):
    """Initial state of ensemble member `index`: one circle of radius 0.3 L,
    noise seed 100 + index."""
    return circle_bilayer(member["N"], member["L"], member["eps"], seed=100 + index)


def psd_mix(N: int = 256, seed: int = 0):
    """The 2048^2 PSD workload's kind of initial data at a smaller size: three
    perturbed circles on a -0.99 background plus a Gaussian random field
    (l = 4 eps, std 1e-3), eps 0.05 and the same h = 16 pi / 2048."""
    eps = 0.05
    L = N * 16 * np.pi / 2048
    kw = dict(N=N, L=L, eps=eps, eta1=1.45, eta2=2.0)
    u = perturbed_circles(N, L, eps, 3, seed=seed, u_bg=-0.99, noise=0.0, r_range=(0.3, 0.6))
    return kw, u + gaussian_random_field(N, L, 4 * eps, 1e-3, seed=seed + 1)


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
