"""The paper's benchmark initial data (Sec. 2.3, eq. dcoef, Table t:Benchmark):
 * the initial masses printed in Table t:Benchmark (6.11, 7.61, 6.93, 6.11,
   6.11), to their printed rounding;
 * mass differences between benchmarks equal |Omega| eps (d1 - d0) / (2 alpha_m(0)^2)
   exactly (the filter keeps the mean);
 * the strip area equals 2 R times the length of Gamma (the area between the
   offset curves of a closed curve whose curvature radius exceeds R);
 * the 512 and 1024 grids are spectral interpolations of the 256 data (equal at
   the shared points)."""
import numpy as np
import pytest

from paper_2006_04784_amd import inputs


def _mass(kw, u0):
    h = kw["L"] / kw["N"]
    return 0.5 * h * h * float(np.sum(u0 + 1.0))


@pytest.fixture(scope="module")
def ics():
    return {name: inputs.paper_initial_data(name) for name in inputs.PAPER_BENCHMARKS}


def test_table_masses(ics):
    for name, (kw, u0) in ics.items():
        assert abs(_mass(kw, u0) - inputs.PAPER_BENCHMARKS[name]["mass"]) <= 0.005, name


def test_mass_differences_are_exact(ics):
    base_kw, base = ics["sub-critical"]
    m0 = _mass(base_kw, base)
    for name, (kw, u0) in ics.items():
        dd = inputs.PAPER_BENCHMARKS[name]["d"] - inputs.PAPER_BENCHMARKS["sub-critical"]["d"]
        pred = 0.5 * inputs.PAPER_L ** 2 * 0.1 * dd / inputs.PAPER_ALPHA0 ** 2
        assert abs(_mass(kw, u0) - m0 - pred) < 1e-10, name


def test_strip_area_is_2R_times_length():
    th = np.linspace(0.0, 2 * np.pi, 200001)
    x, y = inputs.paper_curve(th)
    length = float(np.sum(np.hypot(np.diff(x), np.diff(y))))
    phi = inputs.paper_strip_indicator()
    h = inputs.PAPER_L / inputs.PAPER_N0
    area = h * h * float(np.sum(phi + 1.0)) / 2
    assert abs(area - 2 * inputs.PAPER_R * length) < 2e-3 * area, (area, length)


@pytest.mark.parametrize("N", [512, 1024])
def test_finer_grids_interpolate(ics, N):
    _, u256 = ics["sub-critical"]
    kw, u = inputs.paper_initial_data("sub-critical", N=N)
    s = N // 256
    assert np.max(np.abs(u[::s, ::s] - u256)) < 1e-12
    assert abs(_mass(kw, u) - _mass(dict(kw, N=256), u256)) < 1e-10


def test_defect_onset_from_running_maxima():
    """Sec. 5.1's reading: the onset is the smallest d whose running max of u
    crosses the threshold; the sweep also reports the largest d without a
    defect, which exceeds the onset when the outcome is not monotone in d."""
    from paper_2006_04784_amd import sweeps
    ds = sweeps.paper_d_values()
    assert len(ds) == 206 and ds[0] == 0.7523 and ds[-1] == 0.7728
    assert all(abs(b - a - 1e-4) < 1e-12 for a, b in zip(ds, ds[1:]))
    um = [0.358 if d < 0.7600 else 0.75 for d in ds]
    assert sweeps.onset(ds, um) == (0.76, 0.7599)
    um[ds.index(0.7650)] = 0.357          # one member above the onset without a defect
    assert sweeps.onset(ds, um) == (0.76, 0.765)
    assert sweeps.onset(ds, [0.358] * len(ds)) == (None, 0.7728)
    assert sweeps.onset(ds, [float("nan")] * len(ds)) == (None, 0.7728)
    assert sweeps.onset(ds, [0.9] * len(ds)) == (0.7523, None)


def test_cost_at_error_interpolation():
    """Sec. 5.2's cost at a global error target: going down a scheme's
    sigma_tol sweep, the FFT calls where the error first reaches the target,
    interpolated log-log between the runs on either side of it."""
    from paper_2006_04784_amd import sweeps
    # error = 10 * calls^-1 exactly (a power law): interpolation is exact
    rows = [{"scheme": "imex", "sigma_tol": s, "fft_calls": c, "error": 10.0 / c}
            for s, c in ((1e-4, 1e3), (1e-5, 1e4), (1e-6, 1e5))]
    hit = sweeps.cost_at_error(rows, 2.5e-4)["imex"]
    assert abs(hit["fft_calls"] - 4e4) < 1e-6 * 4e4 and hit["between_sigma_tol"] == (1e-5, 1e-6)
    # the coarsest run already meets the target: its calls, flagged
    assert sweeps.cost_at_error(rows, 2e-2)["imex"]["coarsest_run"]
    # never reached; failed runs (no error) are skipped
    rows.append({"scheme": "psd", "sigma_tol": 1e-3, "failed": "no convergence"})
    rows.append({"scheme": "psd", "sigma_tol": 1e-4, "fft_calls": 10, "error": 0.5})
    res = sweeps.cost_at_error(rows, 1e-6)
    assert res["imex"] is None and res["psd"] is None
    # a non-monotone error curve: the first crossing in sweep order counts
    rows = [{"scheme": "sav", "sigma_tol": s, "fft_calls": c, "error": e}
            for s, c, e in ((1e-4, 100, 1e-2), (1e-5, 200, 1e-3), (1e-6, 400, 2e-3),
                            (1e-7, 800, 1e-4))]
    hit = sweeps.cost_at_error(rows, 5e-3)["sav"]
    assert hit["between_sigma_tol"] == (1e-4, 1e-5) and 100 < hit["fft_calls"] < 200
    assert hit["cheapest_run"] == {"fft_calls": 200, "sigma_tol": 1e-5}
    # cost falling down the sweep: the coarsest run reaches the target, a
    # finer one is cheaper
    rows = [{"scheme": "psd", "sigma_tol": s, "fft_calls": c, "error": e}
            for s, c, e in ((1e-3, 900, 1e-4), (1e-4, 500, 5e-5), (1e-5, 700, 1e-5))]
    hit = sweeps.cost_at_error(rows, 7e-4)["psd"]
    assert hit["coarsest_run"] and hit["fft_calls"] == 900
    assert hit["cheapest_run"] == {"fft_calls": 500, "sigma_tol": 1e-4}
