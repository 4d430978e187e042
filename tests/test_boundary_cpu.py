"""CPU checks of the C ABI library: it loads, exports every function that
include/fch.h declares, and its host-only entry points behave (argument
validation, compiled launch configurations, alpha_m against Table
t:Benchmark, the SAV constants of the documented reading)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fch.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fch_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def fch():
    from paper_2006_04784_amd import fch as F
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("libfch.so not built")
    return F


def test_exports_every_declared_symbol(fch):
    lib = fch.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
        assert n in fch.EXPORTED, n


def test_status_strings(fch):
    for code in range(-6, 1):
        assert fch.lib().fch_status_string(code)


def _prm(fch, **kw):
    base = dict(N=64, L=4 * np.pi, eps=0.1, eta1=1.45, eta2=2.0, p=1, q=0.0, gamma_w=0.3,
                b_minus=-1.0, b_plus=1.0, beta1=2.0, beta2=1.0, zeta=1.1, D0=163.0)
    base.update(kw)
    return fch.fch_params(*[base[k] for k, _ in fch.fch_params._fields_])


def test_alpha_m_table1(fch):
    rows = np.loadtxt(os.path.join(ROOT, "tests", "golden", "table1_alpha_m.txt"))
    for q, eps, alpha in rows:
        assert abs(fch.lib().fch_alpha_m(C.byref(_prm(fch, q=q, eps=eps))) - alpha) < 1e-13


def test_sav_constants_reading(fch):
    # q = 0: min W'' = -1.0075 at u = -0.05, so zeta = 1.1; the C1 box
    # (L = 4 pi, eta2_eff = 0.2) has min (W'^2/2 - eta2 W) ~ -0.0322
    z, d = fch.sav_constants(_prm(fch))
    assert z == pytest.approx(1.1)
    L = 4 * np.pi
    assert d == pytest.approx(L * L * 1.0322, rel=2e-4)


def test_plan_create_rejects_bad_params_before_touching_the_device(fch):
    h = C.c_void_p()
    for kw, code in [(dict(N=48), fch.FCH_E_INVALID), (dict(N=8), fch.FCH_E_UNSUPPORTED),
                     (dict(N=8192), fch.FCH_E_UNSUPPORTED), (dict(L=-1.0), fch.FCH_E_INVALID),
                     (dict(eps=0.0), fch.FCH_E_INVALID), (dict(q=-0.1), fch.FCH_E_INVALID),
                     (dict(eta1=float("nan")), fch.FCH_E_INVALID)]:
        assert fch.lib().fch_plan_create(C.byref(_prm(fch, **kw)), C.byref(h)) == code, kw
    assert fch.lib().fch_plan_create(None, C.byref(h)) == fch.FCH_E_INVALID


def test_compiled_configurations(fch):
    for N in (16, 32, 64, 128, 256, 512, 1024, 2048, 4096):
        rows, cols = fch.config_list(N)
        assert rows and cols, N
        for (R, rE, twl) in rows:
            assert N % rE == 0 and N % (2 * R) == 0 and twl in (0, 1)
            assert rE == N or N >= rE * rE          # radix schedule E ... E
            # LDS: R rows + optional twiddles + reduction scratch <= 160 KiB
            assert 16 * R * (N + N // 8 + 9) + 16 * N * twl + 16 * R * (N // rE) <= 160 * 1024
        for (cE, ctw) in cols:
            assert N % cE == 0 and (cE == N or N >= cE * cE) and ctw in (0, 1)
            assert 2 * 16 * (N + N // 8 + 1) + 16 * N * ctw + 16 * (N // cE) <= 160 * 1024
    assert fch.lib().fch_row_config_count(8192) == 0
    assert fch.lib().fch_col_config_count(100) == 0
    c = fch.fch_launch_cfg()
    assert fch.lib().fch_config_get(1024, 99, 0, C.byref(c)) == fch.FCH_E_UNSUPPORTED


def test_ensemble_create_rejects_bad_options_before_touching_the_device(fch):
    """fch_ensemble_create validates its options and every member before any
    device work: PSD is not batched, ETDRK2 stabilizers must be finite and
    >= 0, t_end > 0, at least two steps, supported grid sizes."""
    arr = (fch.fch_params * 1)(_prm(fch))
    ok = dict(t_end=1.0, max_steps=10, k_first=0.0, umax_t0=0.0, scheme=fch.FCH_IMEX,
              etd=(0.01, 15.0))

    def opts(**kw):
        o = dict(ok, **kw)
        return fch.fch_ensemble_opts(fch.AdaptOpts().c(), o["t_end"], o["max_steps"],
                                     o["k_first"], o["umax_t0"], o["scheme"],
                                     fch.fch_etd_opts(*o["etd"]))

    h = C.c_void_p()
    for kw in (dict(scheme=fch.FCH_PSD), dict(scheme=7), dict(scheme=fch.FCH_ETD, etd=(-1.0, 15.0)),
               dict(scheme=fch.FCH_ETD, etd=(0.01, float("nan"))), dict(t_end=0.0),
               dict(max_steps=1), dict(umax_t0=float("nan"))):
        assert fch.lib().fch_ensemble_create(arr, 1, C.byref(opts(**kw)), C.byref(h)) == \
            fch.FCH_E_INVALID, kw
        assert not h.value
    assert fch.lib().fch_ensemble_create(arr, 0, C.byref(opts()), C.byref(h)) == fch.FCH_E_INVALID
    big = (fch.fch_params * 1)(_prm(fch, N=8192))
    assert fch.lib().fch_ensemble_create(big, 1, C.byref(opts()), C.byref(h)) == \
        fch.FCH_E_UNSUPPORTED


def test_every_entry_point_rejects_null_arguments(fch):
    """Each compute entry point checks its handle and pointers on the host
    before any device work: all-null (and zero-size) arguments return
    FCH_E_INVALID, and the size queries return 0 for a null handle."""
    L = fch.lib()
    sizes = {"fch_plan_workspace_bytes", "fch_ensemble_workspace_bytes",
             "fch_inverse_batch_ws_bytes", "fch_nn_bwd_w_scratch_floats",
             "fch_nn_features_work_doubles"}
    host_only = {"fch_sav_constants", "fch_alpha_m", "fch_row_config_count",
                 "fch_col_config_count", "fch_config_get", "fch_status_string"}
    checked = 0
    for name, (res, args) in fch._SIGS.items():
        if name in host_only:
            continue
        vals = [0 if a in (C.c_int32, C.c_int64, C.c_size_t, C.c_double) else None for a in args]
        r = getattr(L, name)(*vals)
        if name in sizes:
            if args[0] is C.c_void_p:
                assert r == 0, name
        else:
            assert r == fch.FCH_E_INVALID, (name, r)
        checked += 1
    assert checked > 50


def test_tune_cache_reader_tolerates_bad_files(fch, tmp_path):
    """The launch-choice cache reads as empty when missing, unparsable or not
    a mapping, and returns the stored entries otherwise."""
    p = tmp_path / "tune.json"
    assert fch._tune_cache_read(str(p)) == {}
    p.write_text("{broken")
    assert fch._tune_cache_read(str(p)) == {}
    p.write_text("[1, 2]")
    assert fch._tune_cache_read(str(p)) == {}
    p.write_text('{"gfx950|N=256|lib=x": {"config": [4, 8, 0, 4, 0], "us": [1.0, 2.0]}}')
    assert fch._tune_cache_read(str(p))["gfx950|N=256|lib=x"]["config"] == [4, 8, 0, 4, 0]


def test_checkpoint_file_round_trip(fch, tmp_path):
    """save_checkpoint writes exactly the path it is given (no suffix added) and
    load_checkpoint returns the spectra and scalars unchanged."""
    import torch
    a = torch.randn(5, 8, dtype=torch.complex128)
    b = torch.randn(5, 8, dtype=torch.complex128)
    info = {"k_last": 1e-3, "k_next": 1.25e-3, "rs": (3.5, 3.25)}
    path = str(tmp_path / "ckpt")
    fch.save_checkpoint(path, a, b, info, "sav", t=0.125)
    assert os.path.exists(path) and not os.path.exists(path + ".npz")
    x, y, meta = fch.load_checkpoint(path, device="cpu")
    assert torch.equal(x, a) and torch.equal(y, b)
    assert meta == {"scheme": "sav", "k_last": 1e-3, "k_next": 1.25e-3, "rs": [3.5, 3.25],
                    "t": 0.125}


def test_bench_traffic_summaries_name_their_kernels():
    """The committed counter summaries record the kernel each figure was
    taken on, and the bench takes a figure only for that kernel and only on
    the kernel source the counters saw."""
    import importlib.util
    import sys
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    argv, sys.argv = sys.argv, ["bench.py"]
    try:
        spec.loader.exec_module(bench)
    finally:
        sys.argv = argv
    for summary, N in (("pmc_traffic_m1_imex.txt", 1024), ("pmc_traffic_c3_psd.txt", 2048)):
        kv = {}
        for line in open(os.path.join(ROOT, "profiles", summary)):
            m = re.match(r"\s*([a-z_0-9]+)\s*:\s*(.+?)\s*$", line)
            if m:
                kv[m.group(1)] = m.group(2)
        name = kv["row_mu_kernel"]
        m = re.fullmatch(r"fch::k_row<(\d+), (\d+), (\d+), 0, (\d)>", name)
        assert m and int(m.group(1)) == N, name
        cfg = (int(m.group(2)), int(m.group(3)), int(m.group(4)), 4, 0)
        assert bench.row_kernel_name(N, cfg) == name
        other = (cfg[0], cfg[1], 1 - cfg[2], 4, 0)
        assert bench.read_traffic("row_mu", summary, bench.row_kernel_name(N, other)) is None
        got = bench.read_traffic("row_mu", summary, name)
        if kv["kernel_source_sha256"] == bench.kernel_source_hash():
            assert got == float(kv["row_mu_bytes_per_launch"])
        else:
            assert got is None


def test_stored_warm_start_parameters():
    """The stored full-scale parameters of the learned warm start match the
    network's architecture and load without unpickling anything."""
    from paper_2006_04784_amd import nn
    path = os.path.join(ROOT, "paper_2006_04784_amd", "data", "warm_start_c5_full.npz")
    with np.load(path, allow_pickle=False) as z:
        assert tuple(int(c) for c in z["layers"]) == tuple(nn.LAYERS)
        assert int(z["ch"]) == nn.CH and int(z["in_ch"]) == nn.IN_CH
        p = np.asarray(z["params"])
    n = sum(9 * c * nn.CH + c for c in nn.LAYERS)
    assert p.dtype == np.float32 and p.shape == (n,) and np.isfinite(p).all()
    # unused input channels of the first layer stay zero through training
    w0 = p[:9 * nn.LAYERS[0] * nn.CH].reshape(9, nn.LAYERS[0], nn.CH)
    assert not w0[:, :, nn.IN_CH:].any() and w0[:, :, :nn.IN_CH].any()
