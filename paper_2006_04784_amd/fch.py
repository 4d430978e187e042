"""ctypes binding of the HIP library ``libfch.so`` (C ABI in include/fch.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  Spectral
tensors are complex128 of shape (N//2+1, N) (kx-major half spectrum);
physical tensors are float64 of shape (N, N).  Nothing here falls back to a
CPU implementation: a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import json
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# FCH_LIB selects another build of the same sources (the host-sanitized one)
LIB_PATH = os.environ.get("FCH_LIB", os.path.join(HERE, "libfch.so"))
_lib = None

FCH_OK, FCH_E_INVALID, FCH_E_UNSUPPORTED, FCH_E_HIP, FCH_E_NOMEM, FCH_E_NOCONV, FCH_E_NONFINITE = \
    0, -1, -2, -3, -4, -5, -6
FCH_IMEX, FCH_SAV, FCH_PSD, FCH_ETD = 0, 1, 2, 3
# largest N of fch_step_imex_static (FCH_STATIC_MAX_N)
STATIC_MAX_N = 512
# the ETDRK2 split constants used for every simulation of Sec. 3.6
ETD_KAPPA0, ETD_KAPPA2 = 1e-2, 15.0


class FchError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (status %d)" % (msg, code))
        self.code = code


class fch_params(C.Structure):
    _fields_ = [("N", C.c_int32), ("L", C.c_double), ("eps", C.c_double),
                ("eta1", C.c_double), ("eta2", C.c_double), ("p", C.c_int32),
                ("q", C.c_double), ("gamma_w", C.c_double), ("b_minus", C.c_double),
                ("b_plus", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("zeta", C.c_double), ("D0", C.c_double)]


class fch_launch_cfg(C.Structure):
    _fields_ = [("row_R", C.c_int32), ("row_E", C.c_int32), ("row_twl", C.c_int32),
                ("col_E", C.c_int32), ("col_twl", C.c_int32)]


class fch_stats(C.Structure):
    _fields_ = [("fft_calls", C.c_int64), ("launches", C.c_int64), ("psd_iters", C.c_int64),
                ("steps", C.c_int64), ("rejected", C.c_int64)]


class fch_profile(C.Structure):
    _fields_ = [("count", C.c_int64 * 4), ("ms", C.c_double * 4)]


class fch_psd_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("lambda_", C.c_double),
                ("fixed_iters", C.c_int32)]


class fch_psd_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("fft_calls", C.c_int64), ("last_ratio", C.c_double)]


class fch_adapt_opts(C.Structure):
    _fields_ = [("sigma_tol", C.c_double), ("k_min", C.c_double), ("k_max", C.c_double),
                ("rho_s", C.c_double), ("cap", C.c_double)]


class fch_etd_opts(C.Structure):
    _fields_ = [("kappa0", C.c_double), ("kappa2", C.c_double)]


class fch_run_opts(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("adaptive", C.c_int32), ("startup", C.c_int32),
                ("nsteps", C.c_int64), ("k", C.c_double), ("k_prev", C.c_double),
                ("k_first", C.c_double), ("t_end", C.c_double), ("adapt", fch_adapt_opts),
                ("psd", fch_psd_opts), ("etd", fch_etd_opts), ("dyadic", C.c_int32)]


class fch_run_info(C.Structure):
    _fields_ = [("accepted", C.c_int64), ("rejected", C.c_int64), ("psd_iters", C.c_int64),
                ("fft_calls", C.c_int64), ("t", C.c_double), ("k_last", C.c_double),
                ("k_next", C.c_double)]


class fch_ensemble_opts(C.Structure):
    _fields_ = [("adapt", fch_adapt_opts), ("t_end", C.c_double), ("max_steps", C.c_int64),
                ("k_first", C.c_double), ("umax_t0", C.c_double), ("scheme", C.c_int32),
                ("etd", fch_etd_opts)]


class fch_ensemble_info(C.Structure):
    _fields_ = [("attempts", C.c_int64), ("accepted", C.c_int64), ("rejected", C.c_int64),
                ("active", C.c_int32)]


class fch_member_info(C.Structure):
    _fields_ = [("N", C.c_int32), ("done", C.c_int32), ("nonfinite", C.c_int32),
                ("invalid", C.c_int32), ("accepted", C.c_int64), ("rejected", C.c_int64),
                ("t", C.c_double), ("k_last", C.c_double), ("k_next", C.c_double),
                ("err", C.c_double), ("umax", C.c_double), ("r_n", C.c_double),
                ("r_nm1", C.c_double)]


_V = C.c_void_p
_D = C.c_double
_I = C.c_int32
_PD = C.POINTER(C.c_double)
_PI = C.POINTER(C.c_int32)

_SIGS = {
    "fch_sav_constants": (_I, [C.POINTER(fch_params), _PD, _PD]),
    "fch_alpha_m": (_D, [C.POINTER(fch_params)]),
    "fch_plan_create": (_I, [C.POINTER(fch_params), C.POINTER(_V)]),
    "fch_plan_destroy": (_I, [_V]),
    "fch_plan_set_stream": (_I, [_V, _V]),
    "fch_plan_workspace_bytes": (C.c_size_t, [_V]),
    "fch_plan_set_workspace": (_I, [_V, _V, C.c_size_t]),
    "fch_plan_set_config": (_I, [_V, C.POINTER(fch_launch_cfg)]),
    "fch_plan_get_config": (_I, [_V, C.POINTER(fch_launch_cfg)]),
    "fch_plan_set_psd_solve": (_I, [_V, _I, _I]),
    "fch_plan_get_psd_solve": (_I, [_V, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "fch_row_config_count": (_I, [_I]),
    "fch_col_config_count": (_I, [_I]),
    "fch_config_get": (_I, [_I, _I, _I, C.POINTER(fch_launch_cfg)]),
    "fch_autotune": (_I, [_V, _V, _V, _D, _I, C.POINTER(fch_launch_cfg), _PD]),
    "fch_plan_stats": (_I, [_V, C.POINTER(fch_stats)]),
    "fch_plan_reset_stats": (_I, [_V]),
    "fch_plan_profile": (_I, [_V, _I]),
    "fch_forward_batch": (_I, [_V, _I, _V, _V]),
    "fch_inverse_batch_ws_bytes": (C.c_size_t, [_V, _I]),
    "fch_inverse_batch": (_I, [_V, _I, _V, _V, _V, C.c_size_t]),
    "fch_step_imex_dev": (_I, [_V, _V, _V, _V, _V, _V]),
    "fch_step_sav_dev": (_I, [_V, _V, _V, _V, _V, _V, _V, _V]),
    "fch_step_psd_dev": (_I, [_V, _V, _V, _V, _V, _V, _V, _V, _V]),
    "fch_adapt_dt_dev": (_I, [_V, _V, _V, _V, _V, _V, _V, _V, _V, _V]),
    "fch_plan_set_graph": (_I, [_V, _I]),
    "fch_plan_profile_read": (_I, [_V, C.POINTER(fch_profile)]),
    "fch_forward": (_I, [_V, _V, _V]),
    "fch_inverse": (_I, [_V, _V, _V]),
    "fch_chem_potential": (_I, [_V, _V, _V, _PD]),
    "fch_chem_potential_dev": (_I, [_V, _V, _V, _V, _V, _V]),
    "fch_step_imex": (_I, [_V, _V, _V, _D, _D, _V]),
    "fch_step_imex_static": (_I, [_V, _V, _V, _D, _D, _V]),
    "fch_step_etd": (_I, [_V, _V, _V, _D, C.POINTER(fch_etd_opts), _V]),
    "fch_step_etd_dev": (_I, [_V, _V, _V, _V, C.POINTER(fch_etd_opts), _V, _V]),
    "fch_step_sav": (_I, [_V, _V, _V, _D, _D, _D, _D, _V, _PD]),
    "fch_sav_r": (_I, [_V, _V, _PD]),
    "fch_step_psd": (_I, [_V, _V, _V, _D, _D, _V, C.POINTER(fch_psd_opts), _V,
                          C.POINTER(fch_psd_stats)]),
    "fch_adapt_dt": (_I, [_V, _V, _V, _V, _V, _D, _D, C.POINTER(fch_adapt_opts), _V, _PI,
                          _PD, _PD]),
    "fch_rhs": (_I, [_V, _V, _V]),
    "fch_run": (_I, [_V, C.POINTER(fch_run_opts), _V, _V, _PD, C.POINTER(fch_run_info)]),
    "fch_ensemble_create": (_I, [C.POINTER(fch_params), _I, C.POINTER(fch_ensemble_opts),
                                 C.POINTER(_V)]),
    "fch_ensemble_destroy": (_I, [_V]),
    "fch_ensemble_set_stream": (_I, [_V, _V]),
    "fch_ensemble_workspace_bytes": (C.c_size_t, [_V]),
    "fch_ensemble_set_workspace": (_I, [_V, _V, C.c_size_t]),
    "fch_ensemble_load": (_I, [_V, _I, _V]),
    "fch_ensemble_autotune": (_I, [_V, _I]),
    "fch_ensemble_run": (_I, [_V, C.c_int64, _I, _I, C.POINTER(fch_ensemble_info)]),
    "fch_ensemble_step": (_I, [_V, _I, _I]),
    "fch_ensemble_member": (_I, [_V, _I, _V, _PD, C.POINTER(fch_member_info)]),
    "fch_nn_conv_fwd": (_I, [_I, _I, _I, _I, _V, _V, _V, _V, _V, _V, _V]),
    "fch_nn_conv_bwd_data": (_I, [_I, _I, _I, _I, _V, _V, _V, _V, _V, _V]),
    "fch_nn_bwd_w_scratch_floats": (C.c_size_t, [_I, _I, _I]),
    "fch_nn_conv_bwd_w": (_I, [_I, _I, _I, _I, _V, _V, _V, _V, _V]),
    "fch_nn_mse": (_I, [_I, _V, _V, _V, _V, _I, _V]),
    "fch_nn_adam": (_I, [_I, _V, _V, _V, _V, _V, _D, _D, _D, _D, _I, _V]),
    "fch_nn_to_bf16": (_I, [_I, _V, _V, _V]),
    "fch_nn_features_work_doubles": (_I, [_I]),
    "fch_nn_features": (_I, [_I, _I, _I, _V, _V, _V, _V, _V, _V, _V, _V, _V]),
    "fch_nn_guess": (_I, [_I, _I, _I, _V, _V, _V, _V, _V, _V, _V]),
    "fch_nn_reduce": (_I, [_I, _I, _V, _V, _V]),
    "fch_status_string": (C.c_char_p, [_I]),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libfch.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is not built; run __graft_entry__.build()" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(code):
    if code != FCH_OK:
        raise FchError(code, lib().fch_status_string(code).decode())


def _p(t):
    return None if t is None else _V(t.data_ptr())


def sav_constants(prm: fch_params):
    z, d = C.c_double(), C.c_double()
    _check(lib().fch_sav_constants(C.byref(prm), C.byref(z), C.byref(d)))
    return z.value, d.value


_LIB_DIGEST = None


def tune_key(N, device="cuda:0"):
    """Key of a tuned launch choice: the GPU's architecture, the grid size and
    a digest of the library (a rebuilt library tunes again)."""
    global _LIB_DIGEST
    if _LIB_DIGEST is None:
        h = hashlib.sha256()
        with open(LIB_PATH, "rb") as fh:
            for chunk in iter(lambda: fh.read(1 << 20), b""):
                h.update(chunk)
        _LIB_DIGEST = h.hexdigest()[:16]
    props = torch.cuda.get_device_properties(torch.device(device))
    arch = getattr(props, "gcnArchName", "") or props.name
    return "%s|N=%d|lib=%s" % (arch, int(N), _LIB_DIGEST)


def _tune_cache_read(path):
    try:
        with open(path) as fh:
            d = json.load(fh)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def config_list(N: int):
    """Compiled (row variants, column variants) of a grid size: row variants
    as (R, E, twl), column variants as (E, twl)."""
    L = lib()
    rows, cols = [], []
    for i in range(L.fch_row_config_count(N)):
        c = fch_launch_cfg()
        _check(L.fch_config_get(N, i, 0, C.byref(c)))
        rows.append((c.row_R, c.row_E, c.row_twl))
    for j in range(L.fch_col_config_count(N)):
        c = fch_launch_cfg()
        _check(L.fch_config_get(N, 0, j, C.byref(c)))
        cols.append((c.col_E, c.col_twl))
    return rows, cols


@dataclass
class AdaptOpts:
    sigma_tol: float = 1e-5
    k_min: float = 1e-9
    k_max: float = float("inf")
    rho_s: float = 0.9
    cap: float = 1.0 + 2.0 ** 0.5

    def c(self):
        return fch_adapt_opts(self.sigma_tol, self.k_min, self.k_max, self.rho_s, self.cap)


class Plan:
    """A plan for one grid size and parameter set on one device."""

    def __init__(self, N, L, eps, eta1, eta2, p=1, q=0.0, gamma_w=0.3, b_minus=-1.0,
                 b_plus=1.0, beta1=2.0, beta2=1.0, zeta=None, D0=None, device="cuda:0"):
        self.device = torch.device(device)
        prm = fch_params(N, L, eps, eta1, eta2, p, q, gamma_w, b_minus, b_plus, beta1, beta2,
                         0.0, 0.0)
        if zeta is None or D0 is None:
            z, d = sav_constants(prm)
            zeta = z if zeta is None else zeta
            D0 = d if D0 is None else D0
        prm.zeta, prm.D0 = zeta, D0
        self.prm = prm
        self.N, self.H = N, N // 2 + 1
        h = _V()
        with torch.cuda.device(self.device):
            _check(lib().fch_plan_create(C.byref(prm), C.byref(h)))
        self.h = h
        nbytes = lib().fch_plan_workspace_bytes(h)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        _check(lib().fch_plan_set_workspace(h, _V(self.ws.data_ptr() + off), nbytes))

    # -- plumbing -------------------------------------------------------
    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().fch_plan_set_stream(self.h, _V(s)))

    def close(self):
        if getattr(self, "h", None):
            lib().fch_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def spec(self):
        return torch.empty((self.H, self.N), dtype=torch.complex128, device=self.device)

    def phys(self):
        return torch.empty((self.N, self.N), dtype=torch.float64, device=self.device)

    def _chk_spec(self, *ts):
        for t in ts:
            if t is None:
                continue
            if t.dtype != torch.complex128 or tuple(t.shape) != (self.H, self.N) or \
                    not t.is_contiguous() or t.device != self.device:
                raise ValueError("expected contiguous complex128 (%d, %d) on %s" %
                                 (self.H, self.N, self.device))

    def alpha_m(self):
        return lib().fch_alpha_m(C.byref(self.prm))

    def set_config(self, cfg):
        """cfg = (row_R, row_E, row_twl, col_E, col_twl), or None for the default."""
        c = None if cfg is None else fch_launch_cfg(*cfg)
        _check(lib().fch_plan_set_config(self.h, None if c is None else C.byref(c)))

    def set_psd_solve(self, on, grid=0):
        """One-launch PSD solve on (True) or off (separate row and column
        launches); grid > 0: its number of persistent workgroups."""
        _check(lib().fch_plan_set_psd_solve(self.h, int(bool(on)), int(grid)))

    def get_psd_solve(self):
        """(on, grid) of the one-launch PSD solve."""
        on, grid = C.c_int32(), C.c_int32()
        _check(lib().fch_plan_get_psd_solve(self.h, C.byref(on), C.byref(grid)))
        return bool(on.value), grid.value

    def get_config(self):
        c = fch_launch_cfg()
        _check(lib().fch_plan_get_config(self.h, C.byref(c)))
        return (c.row_R, c.row_E, c.row_twl, c.col_E, c.col_twl)

    def autotune(self, uh_n, uh_nm1, k=1e-3, reps=20, cache=None):
        """Pick the fastest compiled row/column variants on the fused IMEX step;
        returns (config, (row_us, col_us)).  cache: path of a JSON file of
        earlier choices keyed by GPU architecture, N and the library's
        contents; a hit sets that choice without timing, a miss tunes and adds
        it (the file is replaced whole, so a reader never sees half of it)."""
        self._chk_spec(uh_n, uh_nm1)
        key = tune_key(self.N, self.device) if cache else None
        if key:
            hit = _tune_cache_read(cache).get(key)
            if hit:
                cfg = tuple(int(x) for x in hit["config"])
                self.set_config(cfg)
                return cfg, tuple(hit["us"])
        c = fch_launch_cfg()
        us = (C.c_double * 2)()
        self._sync_stream()
        _check(lib().fch_autotune(self.h, _p(uh_n), _p(uh_nm1), k, reps, C.byref(c),
                                  C.cast(us, _PD)))
        cfg = (c.row_R, c.row_E, c.row_twl, c.col_E, c.col_twl)
        if key:
            d = _tune_cache_read(cache)
            d[key] = {"config": list(cfg), "us": [us[0], us[1]]}
            tmp = "%s.tmp%d" % (cache, os.getpid())
            with open(tmp, "w") as fh:
                json.dump(d, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return cfg, (us[0], us[1])

    def stats(self):
        s = fch_stats()
        _check(lib().fch_plan_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in fch_stats._fields_}

    def reset_stats(self):
        _check(lib().fch_plan_reset_stats(self.h))

    def set_graph(self, steps):
        """HIP-graph replay of the fixed-step fused IMEX chain, `steps` steps
        per replay (even; 0 disables)."""
        _check(lib().fch_plan_set_graph(self.h, int(steps)))

    def profile(self, enable=True):
        _check(lib().fch_plan_profile(self.h, int(enable)))

    def profile_read(self):
        """Per kernel class: (launch count, summed milliseconds)."""
        pr = fch_profile()
        self._sync_stream()
        _check(lib().fch_plan_profile_read(self.h, C.byref(pr)))
        names = ("row_mu", "col_fused", "col_one_way", "transform")
        return {n: (pr.count[i], pr.ms[i]) for i, n in enumerate(names)}

    # -- calls (same names as the C ABI, minus the prefix) -----------------
    def forward(self, u, out=None):
        if u.dtype != torch.float64 or tuple(u.shape) != (self.N, self.N) or not u.is_contiguous():
            raise ValueError("expected contiguous float64 (N, N)")
        out = self.spec() if out is None else out
        self._sync_stream()
        _check(lib().fch_forward(self.h, _p(u), _p(out)))
        return out

    def inverse(self, uh, out=None):
        self._chk_spec(uh)
        out = self.phys() if out is None else out
        self._sync_stream()
        _check(lib().fch_inverse(self.h, _p(uh), _p(out)))
        return out

    def forward_batch(self, u, out=None):
        """u: contiguous float64 (B, N, N) -> (B, N/2+1, N) complex128 half spectra."""
        if u.dtype != torch.float64 or u.dim() != 3 or tuple(u.shape[1:]) != (self.N, self.N) \
                or not u.is_contiguous() or u.device != self.device:
            raise ValueError("expected contiguous float64 (B, N, N) on %s" % self.device)
        B = int(u.shape[0])
        if out is None:
            out = torch.empty((B, self.H, self.N), dtype=torch.complex128, device=self.device)
        elif out.dtype != torch.complex128 or tuple(out.shape) != (B, self.H, self.N) or \
                not out.is_contiguous() or out.device != self.device:
            raise ValueError("expected contiguous complex128 (B, %d, %d)" % (self.H, self.N))
        self._sync_stream()
        _check(lib().fch_forward_batch(self.h, B, _p(u), _p(out)))
        return out

    def lib_inverse_batch_ws_bytes(self, batch):
        return int(lib().fch_inverse_batch_ws_bytes(self.h, int(batch)))

    def inverse_batch(self, uh, out=None, ws=None):
        """uh: contiguous complex128 (B, N/2+1, N) -> (B, N, N) float64.  ws: optional
        device workspace (uint8 tensor) of fch_inverse_batch_ws_bytes bytes."""
        if uh.dtype != torch.complex128 or uh.dim() != 3 or tuple(uh.shape[1:]) != (self.H, self.N) \
                or not uh.is_contiguous() or uh.device != self.device:
            raise ValueError("expected contiguous complex128 (B, %d, %d)" % (self.H, self.N))
        B = int(uh.shape[0])
        nb = int(lib().fch_inverse_batch_ws_bytes(self.h, B))
        if ws is None:
            ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        if out is None:
            out = torch.empty((B, self.N, self.N), dtype=torch.float64, device=self.device)
        elif out.dtype != torch.float64 or tuple(out.shape) != (B, self.N, self.N) or \
                not out.is_contiguous() or out.device != self.device:
            raise ValueError("expected contiguous float64 (B, N, N)")
        self._sync_stream()
        _check(lib().fch_inverse_batch(self.h, B, _p(uh), _p(out), _p(ws),
                                       ws.numel() * ws.element_size()))
        return out

    def chem_potential(self, uh, out=None, energy=False):
        self._chk_spec(uh)
        out = self.spec() if out is None else out
        e = C.c_double()
        self._sync_stream()
        _check(lib().fch_chem_potential(self.h, _p(uh), _p(out), C.byref(e) if energy else None))
        return (out, e.value) if energy else out

    def chem_potential_dev(self, uh, out=None, mu_phys=None, energy_dev=None, status_dev=None):
        """fch_chem_potential_dev: mu's half spectrum, and optionally mu on the
        grid (float64 (N, N)), the energy (float64 (1,)) and a status (int32
        (1,)), all in device memory."""
        self._chk_spec(uh)
        out = self.spec() if out is None else out
        if mu_phys is not None and (mu_phys.dtype != torch.float64 or
                                    tuple(mu_phys.shape) != (self.N, self.N) or
                                    not mu_phys.is_contiguous() or mu_phys.device != self.device):
            raise ValueError("mu_phys: contiguous float64 (N, N)")
        if energy_dev is not None:
            self._chk_dev(energy_dev, 1, torch.float64)
        if status_dev is not None:
            self._chk_dev(status_dev, 1, torch.int32)
        self._sync_stream()
        _check(lib().fch_chem_potential_dev(self.h, _p(uh), _p(out), _p(mu_phys),
                                            _p(energy_dev), _p(status_dev)))
        return out

    def rhs(self, uh, out=None):
        self._chk_spec(uh)
        out = self.spec() if out is None else out
        self._sync_stream()
        _check(lib().fch_rhs(self.h, _p(uh), _p(out)))
        return out

    def step_imex(self, uh_n, uh_nm1, k_np1, k_n, out=None):
        self._chk_spec(uh_n, uh_nm1)
        out = self.spec() if out is None else out
        self._sync_stream()
        _check(lib().fch_step_imex(self.h, _p(uh_n), _p(uh_nm1), k_np1, k_n, _p(out)))
        return out

    def step_imex_static(self, uh_n, uh_nm1, k_np1, k_n, out=None):
        """fch_step_imex_static: the IMEX step with the library's own scratch
        (N <= STATIC_MAX_N); needs no workspace and allocates nothing."""
        self._chk_spec(uh_n, uh_nm1)
        out = self.spec() if out is None else out
        self._sync_stream()
        _check(lib().fch_step_imex_static(self.h, _p(uh_n), _p(uh_nm1), k_np1, k_n, _p(out)))
        return out

    def step_etd(self, uh_n, k, F_n=None, kappa0=ETD_KAPPA0, kappa2=ETD_KAPPA2, out=None):
        """One ETDRK2 step (fch_step_etd); F_n (optional) = F(u^n) = Lap mu(u^n)."""
        self._chk_spec(uh_n, F_n)
        out = self.spec() if out is None else out
        o = fch_etd_opts(kappa0, kappa2)
        self._sync_stream()
        _check(lib().fch_step_etd(self.h, _p(uh_n), _p(F_n), k, C.byref(o), _p(out)))
        return out

    def sav_r(self, uh):
        self._chk_spec(uh)
        r = C.c_double()
        self._sync_stream()
        _check(lib().fch_sav_r(self.h, _p(uh), C.byref(r)))
        return r.value

    def step_sav(self, uh_n, uh_nm1, r_n, r_nm1, k_np1, k_n, out=None):
        self._chk_spec(uh_n, uh_nm1)
        out = self.spec() if out is None else out
        r = C.c_double()
        self._sync_stream()
        _check(lib().fch_step_sav(self.h, _p(uh_n), _p(uh_nm1), r_n, r_nm1, k_np1, k_n, _p(out),
                                  C.byref(r)))
        return out, r.value

    def step_psd(self, uh_n, uh_nm1, k_np1, k_n, guess=None, tol=1e-10, max_iter=1000,
                 lam=0.0, fixed_iters=0, out=None, raise_noconv=True):
        self._chk_spec(uh_n, uh_nm1, guess)
        out = self.spec() if out is None else out
        o = fch_psd_opts(tol, max_iter, lam, fixed_iters)
        st = fch_psd_stats()
        self._sync_stream()
        code = lib().fch_step_psd(self.h, _p(uh_n), _p(uh_nm1), k_np1, k_n, _p(guess),
                                  C.byref(o), _p(out), C.byref(st))
        if code != FCH_E_NOCONV or raise_noconv:
            _check(code)
        return out, {"iters": st.iters, "fft_calls": st.fft_calls,
                     "last_ratio": st.last_ratio, "status": code}

    def adapt_dt(self, uh_trial, uh_n, F_n, F_nm1, k_trial, k_n, opts: AdaptOpts = None,
                 out=None):
        self._chk_spec(uh_trial, uh_n, F_n, F_nm1)
        out = self.spec() if out is None else out
        o = (opts or AdaptOpts()).c()
        acc, kn, err = C.c_int32(), C.c_double(), C.c_double()
        self._sync_stream()
        _check(lib().fch_adapt_dt(self.h, _p(uh_trial), _p(uh_n), _p(F_n), _p(F_nm1), k_trial,
                                  k_n, C.byref(o), _p(out), C.byref(acc), C.byref(kn),
                                  C.byref(err)))
        return out, bool(acc.value), kn.value, err.value

    # -- device-scalar (graph-capturable) steps: k_dev etc. are device tensors
    def _chk_dev(self, t, n, dtype):
        if t is None or t.dtype != dtype or t.numel() < n or not t.is_contiguous() or \
                t.device != self.device:
            raise ValueError("expected a contiguous %s device tensor of >= %d values" % (dtype, n))

    def step_imex_dev(self, uh_n, uh_nm1, k_dev, out, status_dev=None):
        self._chk_spec(uh_n, uh_nm1, out)
        self._chk_dev(k_dev, 2, torch.float64)
        if status_dev is not None:
            self._chk_dev(status_dev, 1, torch.int32)
        self._sync_stream()
        _check(lib().fch_step_imex_dev(self.h, _p(uh_n), _p(uh_nm1), _p(k_dev), _p(out),
                                       _p(status_dev)))
        return out

    def step_sav_dev(self, uh_n, uh_nm1, r_dev, k_dev, out, r_np1_dev, status_dev=None):
        self._chk_spec(uh_n, uh_nm1, out)
        self._chk_dev(k_dev, 2, torch.float64)
        self._chk_dev(r_dev, 2, torch.float64)
        self._chk_dev(r_np1_dev, 1, torch.float64)
        if status_dev is not None:
            self._chk_dev(status_dev, 1, torch.int32)
        self._sync_stream()
        _check(lib().fch_step_sav_dev(self.h, _p(uh_n), _p(uh_nm1), _p(r_dev), _p(k_dev),
                                      _p(out), _p(r_np1_dev), _p(status_dev)))
        return out

    def step_psd_dev(self, uh_n, uh_nm1, k_dev, out, iters_dev, status_dev=None, guess=None,
                     tol=1e-10, max_iter=1000, lam=0.0, fixed_iters=0):
        self._chk_spec(uh_n, uh_nm1, out, guess)
        self._chk_dev(k_dev, 2, torch.float64)
        self._chk_dev(iters_dev, 1, torch.int32)
        if status_dev is not None:
            self._chk_dev(status_dev, 1, torch.int32)
        o = fch_psd_opts(tol, max_iter, lam, fixed_iters)
        self._sync_stream()
        _check(lib().fch_step_psd_dev(self.h, _p(uh_n), _p(uh_nm1), _p(k_dev), _p(guess),
                                      C.byref(o), _p(out), _p(iters_dev), _p(status_dev)))
        return out

    def step_etd_dev(self, uh_n, k_dev, out, F_n=None, status_dev=None, kappa0=ETD_KAPPA0,
                     kappa2=ETD_KAPPA2):
        self._chk_spec(uh_n, F_n, out)
        self._chk_dev(k_dev, 1, torch.float64)
        if status_dev is not None:
            self._chk_dev(status_dev, 1, torch.int32)
        o = fch_etd_opts(kappa0, kappa2)
        self._sync_stream()
        _check(lib().fch_step_etd_dev(self.h, _p(uh_n), _p(F_n), _p(k_dev), C.byref(o),
                                      _p(out), _p(status_dev)))
        return out

    def adapt_dt_dev(self, uh_trial, uh_n, F_n, F_nm1, k_dev, out, out_dev, status_dev=None,
                     opts: AdaptOpts = None):
        self._chk_spec(uh_trial, uh_n, F_n, F_nm1, out)
        self._chk_dev(k_dev, 2, torch.float64)
        self._chk_dev(out_dev, 3, torch.float64)
        if status_dev is not None:
            self._chk_dev(status_dev, 1, torch.int32)
        o = (opts or AdaptOpts()).c()
        self._sync_stream()
        _check(lib().fch_adapt_dt_dev(self.h, _p(uh_trial), _p(uh_n), _p(F_n), _p(F_nm1),
                                      _p(k_dev), C.byref(o), _p(out), _p(out_dev),
                                      _p(status_dev)))
        return out

    def resume(self, uh_n, uh_nm1, meta, **kw):
        """Continues a run saved by save_checkpoint (load_checkpoint's meta):
        fch_run without the startup step, from its next trial step, its last
        accepted step and (SAV) its r values; kw as for run (adaptive,
        nsteps, t_end, adapt, ...).  The info's t counts from the resume."""
        args = dict(k=meta["k_next"], k_prev=meta["k_last"], rs=tuple(meta["rs"]))
        args.update(kw)
        return self.run(uh_n, uh_nm1, scheme=meta["scheme"], startup=False, **args)

    def run(self, uh_n, uh_nm1, scheme="imex", adaptive=False, startup=True, nsteps=0, k=1e-3,
            k_prev=0.0, k_first=0.0, t_end=0.0, adapt: AdaptOpts = None, psd_tol=1e-10,
            psd_max_iter=1000, psd_lambda=0.0, rs=None, kappa0=ETD_KAPPA0, kappa2=ETD_KAPPA2,
            dyadic=False):
        """fch_run; dyadic: nested factor-of-two step sizes (adaptive runs)."""
        self._chk_spec(uh_n, uh_nm1)
        sch = {"imex": FCH_IMEX, "sav": FCH_SAV, "psd": FCH_PSD, "etd": FCH_ETD}[scheme]
        o = fch_run_opts(sch, int(adaptive), int(startup), nsteps, k, k_prev, k_first, t_end,
                         (adapt or AdaptOpts()).c(),
                         fch_psd_opts(psd_tol, psd_max_iter, psd_lambda, 0),
                         fch_etd_opts(kappa0, kappa2), int(dyadic))
        r = (C.c_double * 2)(*(rs if rs is not None else (0.0, 0.0)))
        info = fch_run_info()
        self._sync_stream()
        _check(lib().fch_run(self.h, C.byref(o), _p(uh_n), _p(uh_nm1),
                             C.cast(r, _PD), C.byref(info)))
        d = {k_: getattr(info, k_) for k_, _ in fch_run_info._fields_}
        d["rs"] = (r[0], r[1])
        return d


def save_checkpoint(path, uh_n, uh_nm1, info, scheme, t=0.0):
    """Writes what a run of `scheme` needs to continue where fch_run left it
    (info: its returned dict): u^n and u^{n-1} (half spectra), the last
    accepted and the next trial step, SAV's r^n and r^{n-1}, and the elapsed
    time t, as one .npz holding only arrays (readable without unpickling)."""
    meta = {"scheme": scheme, "k_last": float(info["k_last"]), "k_next": float(info["k_next"]),
            "rs": [float(x) for x in info.get("rs", (0.0, 0.0))], "t": float(t)}
    with open(path, "wb") as fh:  # (a path given to savez would gain a .npz suffix)
        np.savez(fh, uh_n=uh_n.detach().cpu().numpy(), uh_nm1=uh_nm1.detach().cpu().numpy(),
                 meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


def load_checkpoint(path, device="cuda:0"):
    """(u^n, u^{n-1}, meta) of save_checkpoint, the spectra on `device`."""
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(bytes(z["meta"]).decode())
        dev = torch.device(device)
        return (torch.from_numpy(z["uh_n"]).to(dev), torch.from_numpy(z["uh_nm1"]).to(dev),
                meta)


class Ensemble:
    """Batched adaptive runs (fch_ensemble_* of the C ABI), one scheme for every member:
    "imex" (BDF2 IMEX), "sav" (BDF2 SAV) or "etd" (ETDRK2 with stabilizers kappa0, kappa2).

    members: list of dicts of Plan keyword arguments (N, L, eps, eta1, eta2, ...)."""

    def __init__(self, members, adapt: AdaptOpts = None, t_end=1.0, max_steps=1000, k_first=0.0,
                 device="cuda:0", umax_t0=0.0, scheme="imex", kappa0=None, kappa2=None):
        self.device = torch.device(device)
        prms = []
        for kw in members:
            kw = dict(kw)
            prm = fch_params(kw["N"], kw["L"], kw["eps"], kw["eta1"], kw["eta2"], kw.get("p", 1),
                             kw.get("q", 0.0), kw.get("gamma_w", 0.3), kw.get("b_minus", -1.0),
                             kw.get("b_plus", 1.0), kw.get("beta1", 2.0), kw.get("beta2", 1.0),
                             0.0, 0.0)
            z, d = sav_constants(prm)
            prm.zeta, prm.D0 = kw.get("zeta", z), kw.get("D0", d)
            prms.append(prm)
        arr = (fch_params * len(prms))(*prms)
        self.Ns = [m["N"] for m in members]
        self.max_steps = max_steps
        schemes = {"imex": FCH_IMEX, "sav": FCH_SAV, "etd": FCH_ETD}
        if scheme not in schemes:
            raise ValueError("ensemble scheme must be one of %s" % sorted(schemes))
        etd = fch_etd_opts(ETD_KAPPA0 if kappa0 is None else kappa0,
                           ETD_KAPPA2 if kappa2 is None else kappa2)
        opts = fch_ensemble_opts((adapt or AdaptOpts()).c(), t_end, max_steps, k_first, umax_t0,
                                 schemes[scheme], etd)
        h = _V()
        with torch.cuda.device(self.device):
            _check(lib().fch_ensemble_create(arr, len(prms), C.byref(opts), C.byref(h)))
        self.h = h
        nbytes = lib().fch_ensemble_workspace_bytes(h)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        _check(lib().fch_ensemble_set_workspace(h, _V(self.ws.data_ptr() + off), nbytes))

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().fch_ensemble_set_stream(self.h, _V(s)))

    def close(self):
        if getattr(self, "h", None):
            lib().fch_ensemble_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, i, u0):
        N = self.Ns[i]
        if u0.dtype != torch.float64 or tuple(u0.shape) != (N, N) or not u0.is_contiguous():
            raise ValueError("expected contiguous float64 (N, N) for member %d" % i)
        self._sync_stream()
        _check(lib().fch_ensemble_load(self.h, i, _p(u0)))

    def autotune(self, reps=10):
        self._sync_stream()
        _check(lib().fch_ensemble_autotune(self.h, reps))

    def step(self, attempts=1, use_graph=True):
        """Queues attempts on the device without waiting (fch_ensemble_step)."""
        self._sync_stream()
        _check(lib().fch_ensemble_step(self.h, int(attempts), int(use_graph)))

    def run(self, max_attempts=100000, sync_every=50, use_graph=True):
        info = fch_ensemble_info()
        self._sync_stream()
        _check(lib().fch_ensemble_run(self.h, max_attempts, sync_every, int(use_graph),
                                      C.byref(info)))
        return {k: getattr(info, k) for k, _ in fch_ensemble_info._fields_}

    def member(self, i, state=True, klog=True):
        import numpy as np
        N = self.Ns[i]
        uh = torch.empty((N // 2 + 1, N), dtype=torch.complex128, device=self.device) \
            if state else None
        log = np.zeros(self.max_steps) if klog else None
        info = fch_member_info()
        self._sync_stream()
        _check(lib().fch_ensemble_member(self.h, i, _p(uh),
                                         log.ctypes.data_as(_PD) if klog else None,
                                         C.byref(info)))
        d = {k: getattr(info, k) for k, _ in fch_member_info._fields_}
        if klog:
            log = log[:min(d["accepted"], self.max_steps)]
        return uh, log, d
