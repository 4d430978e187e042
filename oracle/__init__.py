"""Plain FP64 CPU oracle for the FCH pseudo-spectral BDF2 path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of ``bench.py`` import this package; the product library
(``paper_2006_04784_amd``) never does, and the two share no code.

The arithmetic lives in ``fch_oracle.c`` (plain C99 with complex.h, its own
naive DFT and radix-2 FFT); this module only loads the shared object and
marshals numpy arrays.  Spectra use the numpy ``rfft2`` layout
``uh[ky, kx]`` with shape (N, N//2+1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fch_oracle.c")
_SRC_NN = os.path.join(_HERE, "nn_oracle.c")
_LIB_DEFAULT = os.path.join(_HERE, "liboracle.so")
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
# FCH_ORACLE_LIB selects another build of the same sources (the sanitized one)
_LIB_PATH = os.environ.get("FCH_ORACLE_LIB", _LIB_DEFAULT)
_lib = None
_CLANG = "/opt/rocm/llvm/bin/clang"


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (-O3, OpenMP over independent lines).
    sanitize: a separate liboracle_san.so with AddressSanitizer and
    UndefinedBehaviorSanitizer, built with the ROCm clang so that it shares
    one sanitizer runtime with the sanitized host code of the HIP library
    (no OpenMP)."""
    if sanitize:
        tmp = _LIB_SAN + ".tmp%d" % os.getpid()
        cmd = [_CLANG, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", "-shared-libsan", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-o", tmp, _SRC, _SRC_NN, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_SAN)
        return _LIB_SAN
    if force or not os.path.exists(_LIB_DEFAULT):
        tmp = _LIB_DEFAULT + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-o", tmp, _SRC, _SRC_NN, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_DEFAULT)
    return _LIB_DEFAULT


class Params(C.Structure):
    _fields_ = [("N", C.c_int), ("L", C.c_double), ("eps", C.c_double),
                ("eta1", C.c_double), ("eta2", C.c_double), ("p", C.c_int),
                ("q", C.c_double), ("gamma_w", C.c_double),
                ("b_minus", C.c_double), ("b_plus", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double),
                ("zeta", C.c_double), ("D0", C.c_double)]


@dataclass
class Model:
    """Model and discretization parameters (paper Table t:Benchmark notation)."""
    N: int
    L: float
    eps: float
    eta1: float
    eta2: float
    p: int = 1
    q: float = 0.0
    gamma_w: float = 0.3
    b_minus: float = -1.0
    b_plus: float = 1.0
    beta1: float = 2.0
    beta2: float = 1.0
    zeta: float = 1.1
    D0: float = 0.0

    def c(self) -> Params:
        return Params(self.N, self.L, self.eps, self.eta1, self.eta2, self.p, self.q,
                      self.gamma_w, self.b_minus, self.b_plus, self.beta1, self.beta2,
                      self.zeta, self.D0)


_D = C.POINTER(C.c_double)
_P = C.POINTER(Params)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = C.CDLL(_LIB_PATH)
    sig = {
        "oracle_dft_1d": (None, [C.c_int, _D, _D, C.c_int]),
        "oracle_fft_1d": (C.c_int, [C.c_int, _D, C.c_int]),
        "oracle_dft2_brute": (None, [C.c_int, _D, _D]),
        "oracle_r2c": (C.c_int, [C.c_int, _D, _D, C.c_int]),
        "oracle_c2r": (C.c_int, [C.c_int, _D, _D, C.c_int]),
        "oracle_set_threads": (None, [C.c_int]),
        "oracle_well": (None, [_P, C.c_int, _D, _D, _D, _D]),
        "oracle_alpha_m": (C.c_double, [_P]),
        "oracle_laplacian": (None, [_P, _D, _D]),
        "oracle_mu": (C.c_int, [_P, _D, _D]),
        "oracle_F": (C.c_int, [_P, _D, _D]),
        "oracle_energy": (C.c_double, [_P, _D]),
        "oracle_mass": (C.c_double, [_P, _D]),
        "oracle_E1": (C.c_double, [_P, _D]),
        "oracle_V": (C.c_int, [_P, _D, _D]),
        "oracle_E_aux": (C.c_double, [_P, _D, _D, C.c_double, C.c_double]),
        "oracle_inner": (C.c_double, [_P, _D, _D]),
        "oracle_bdf2_coef": (None, [C.c_double, C.c_double, _D, _D, _D]),
        "oracle_am3_weights": (None, [C.c_double, C.c_double, _D, _D, _D]),
        "oracle_imex_step": (C.c_int, [_P, _D, _D, C.c_double, C.c_double, _D, _D]),
        "oracle_sav_step": (C.c_int, [_P, _D, _D, C.c_double, C.c_double, C.c_double,
                                      C.c_double, _D, _D, _D, _D, _D]),
        "oracle_psd_step": (C.c_int, [_P, _D, _D, C.c_double, C.c_double, _D, _D,
                                      C.c_double, C.c_int, C.c_double, C.c_int, _D,
                                      C.POINTER(C.c_int), _D]),
        "oracle_lambda_table": (C.c_double, [C.c_double, C.c_double]),
        "oracle_am3_error": (C.c_double, [_P, _D, _D, _D, _D, _D, C.c_double, C.c_double]),
        "oracle_adapt_decide": (None, [C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.c_double, C.c_double, C.c_double,
                                       C.POINTER(C.c_int), _D]),
        "oracle_etd_phi": (None, [C.c_double, _D, _D, _D]),
        "oracle_etd_step": (C.c_int, [_P, _D, C.c_double, C.c_double, C.c_double, _D, _D, _D,
                                      _D]),
        "nn_bf16": (C.c_double, [C.c_double]),
        "nn_conv_fwd": (None, [C.c_int, C.c_int, C.c_int, C.c_int, _D, _D, _D, _D, _D, _D,
                               C.c_int]),
        "nn_conv_bwd_data": (None, [C.c_int, C.c_int, C.c_int, C.c_int, _D, _D, _D, _D,
                                    C.c_int]),
        "nn_conv_bwd_w": (None, [C.c_int, C.c_int, C.c_int, C.c_int, _D, _D, _D, _D]),
        "nn_mse": (C.c_double, [C.c_long, _D, _D, _D, C.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _cplx(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _real(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


# ---- transforms ----------------------------------------------------------
def dft_1d(x, sign=-1):
    x = _cplx(x)
    out = np.empty_like(x)
    _load().oracle_dft_1d(x.size, _ptr(x.view(np.float64)), _ptr(out.view(np.float64)), sign)
    return out


def fft_1d(x, sign=-1):
    x = _cplx(x).copy()
    rc = _load().oracle_fft_1d(x.size, _ptr(x.view(np.float64)), sign)
    if rc:
        raise ValueError("length must be a power of two")
    return x


def dft2_brute(u):
    u = _real(u)
    N = u.shape[0]
    out = np.empty((N, N // 2 + 1), np.complex128)
    _load().oracle_dft2_brute(N, _ptr(u), _ptr(out.view(np.float64)))
    return out


def r2c(u, method=1):
    u = _real(u)
    N = u.shape[0]
    out = np.empty((N, N // 2 + 1), np.complex128)
    if _load().oracle_r2c(N, _ptr(u), _ptr(out.view(np.float64)), method):
        raise ValueError("bad size for method")
    return out


def c2r(uh, method=1):
    uh = _cplx(uh)
    N = uh.shape[0]
    out = np.empty((N, N), np.float64)
    if _load().oracle_c2r(N, _ptr(uh.view(np.float64)), _ptr(out), method):
        raise ValueError("bad size for method")
    return out


# ---- model ---------------------------------------------------------------
def well(m: Model, u):
    u = _real(u)
    W = np.empty_like(u)
    W1 = np.empty_like(u)
    W2 = np.empty_like(u)
    _load().oracle_well(C.byref(m.c()), u.size, _ptr(u), _ptr(W), _ptr(W1), _ptr(W2))
    return W, W1, W2


def alpha_m(m: Model) -> float:
    return _load().oracle_alpha_m(C.byref(m.c()))


def laplacian(m: Model, u):
    u = _real(u)
    out = np.empty_like(u)
    _load().oracle_laplacian(C.byref(m.c()), _ptr(u), _ptr(out))
    return out


def _spec_op(fn, m, uh):
    uh = _cplx(uh)
    out = np.empty_like(uh)
    rc = fn(C.byref(m.c()), _ptr(uh.view(np.float64)), _ptr(out.view(np.float64)))
    if rc:
        raise RuntimeError("oracle error %d" % rc)
    return out


def mu(m: Model, uh):
    return _spec_op(_load().oracle_mu, m, uh)


def F(m: Model, uh):
    return _spec_op(_load().oracle_F, m, uh)


def V(m: Model, uh):
    return _spec_op(_load().oracle_V, m, uh)


def energy(m: Model, uh) -> float:
    uh = _cplx(uh)
    return _load().oracle_energy(C.byref(m.c()), _ptr(uh.view(np.float64)))


def mass(m: Model, uh) -> float:
    uh = _cplx(uh)
    return _load().oracle_mass(C.byref(m.c()), _ptr(uh.view(np.float64)))


def E1(m: Model, uh) -> float:
    uh = _cplx(uh)
    return _load().oracle_E1(C.byref(m.c()), _ptr(uh.view(np.float64)))


def E_aux(m: Model, uh_n, uh_nm1, r_n, r_nm1) -> float:
    a, b = _cplx(uh_n), _cplx(uh_nm1)
    return _load().oracle_E_aux(C.byref(m.c()), _ptr(a.view(np.float64)),
                                _ptr(b.view(np.float64)), r_n, r_nm1)


def inner(m: Model, fh, gh) -> float:
    a, b = _cplx(fh), _cplx(gh)
    return _load().oracle_inner(C.byref(m.c()), _ptr(a.view(np.float64)),
                                _ptr(b.view(np.float64)))


# ---- time stepping -------------------------------------------------------
def bdf2_coef(k_np1, k_n):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _load().oracle_bdf2_coef(k_np1, k_n, C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def am3_weights(k_np1, k_n):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _load().oracle_am3_weights(k_np1, k_n, C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def _opt(a):
    return None if a is None else _cplx(a)


def imex_step(m: Model, uh_n, uh_nm1, k_np1, k_n, fh=None):
    un = _cplx(uh_n)
    um = _cplx(uh_nm1 if uh_nm1 is not None else uh_n)
    f = _opt(fh)
    out = np.empty_like(un)
    _load().oracle_imex_step(C.byref(m.c()), _ptr(un.view(np.float64)), _ptr(um.view(np.float64)),
                             k_np1, k_n, None if f is None else _ptr(f.view(np.float64)),
                             _ptr(out.view(np.float64)))
    return out


def sav_step(m: Model, uh_n, uh_nm1, r_n, r_nm1, k_np1, k_n, fh=None, want_q=False):
    un = _cplx(uh_n)
    um = _cplx(uh_nm1 if uh_nm1 is not None else uh_n)
    f = _opt(fh)
    out = np.empty_like(un)
    qh = np.empty_like(un)
    r = C.c_double()
    s = C.c_double()
    rc = _load().oracle_sav_step(C.byref(m.c()), _ptr(un.view(np.float64)),
                                 _ptr(um.view(np.float64)), r_n, r_nm1, k_np1, k_n,
                                 None if f is None else _ptr(f.view(np.float64)),
                                 _ptr(out.view(np.float64)), C.byref(r), C.byref(s),
                                 _ptr(qh.view(np.float64)))
    if rc:
        raise RuntimeError("SAV: E1 + D0 <= 0 (rc=%d)" % rc)
    if want_q:
        return out, r.value, s.value, qh
    return out, r.value


def psd_step(m: Model, uh_n, uh_nm1, k_np1, k_n, guess=None, fh=None, tol=1e-10,
             max_iter=1000, lam=0.0, fixed_iters=0):
    """Returns (u^{n+1} spectrum, iterations, last ratio, rc) with rc 0 on
    convergence and 1 when max_iter was reached."""
    un = _cplx(uh_n)
    um = _cplx(uh_nm1 if uh_nm1 is not None else uh_n)
    g = _opt(guess)
    f = _opt(fh)
    out = np.empty_like(un)
    it = C.c_int()
    ratio = C.c_double()
    rc = _load().oracle_psd_step(C.byref(m.c()), _ptr(un.view(np.float64)),
                                 _ptr(um.view(np.float64)), k_np1, k_n,
                                 None if g is None else _ptr(g.view(np.float64)),
                                 None if f is None else _ptr(f.view(np.float64)),
                                 tol, max_iter, lam, fixed_iters, _ptr(out.view(np.float64)),
                                 C.byref(it), C.byref(ratio))
    if rc < 0:
        raise ValueError("PSD: no lambda for this q; pass lam explicitly")
    return out, it.value, ratio.value, rc


def lambda_table(q, k) -> float:
    return _load().oracle_lambda_table(q, k)


def am3_error(m: Model, uh_trial, uh_n, F_trial, F_n, F_nm1, k_trial, k_n) -> float:
    arrs = [_cplx(x) for x in (uh_trial, uh_n, F_trial, F_n, F_nm1)]
    return _load().oracle_am3_error(C.byref(m.c()), *[_ptr(a.view(np.float64)) for a in arrs],
                                    k_trial, k_n)


def adapt_decide(e, k_trial, sigma_tol, k_min, k_max, rho_s=0.9, cap=1.0 + 2.0 ** 0.5):
    acc = C.c_int()
    kn = C.c_double()
    _load().oracle_adapt_decide(e, k_trial, sigma_tol, k_min, k_max, rho_s, cap,
                                C.byref(acc), C.byref(kn))
    return bool(acc.value), kn.value


# the constants of eq. ETD-L used for every simulation of Sec. 3.6
KAPPA0, KAPPA2 = 1e-2, 15.0


def etd_phi(z):
    """(e^z, (e^z - 1)/z, (e^z - 1 - z)/z^2) at a real z."""
    p0, p1, p2 = C.c_double(), C.c_double(), C.c_double()
    _load().oracle_etd_phi(float(z), C.byref(p0), C.byref(p1), C.byref(p2))
    return p0.value, p1.value, p2.value


def etd_step(m: Model, uh_n, k, kappa0=KAPPA0, kappa2=KAPPA2, fh_n=None, fh_np1=None,
             want_stage=False):
    """One ETDRK2 step (eqs. ETDRK1, ETDRK2, ETD-L); returns u^{n+1} (and the
    ETDRK1 stage u~ if want_stage)."""
    un = _cplx(uh_n)
    f0, f1 = _opt(fh_n), _opt(fh_np1)
    out = np.empty_like(un)
    st = np.empty_like(un)
    rc = _load().oracle_etd_step(C.byref(m.c()), _ptr(un.view(np.float64)), k, kappa0, kappa2,
                                 None if f0 is None else _ptr(f0.view(np.float64)),
                                 None if f1 is None else _ptr(f1.view(np.float64)),
                                 _ptr(out.view(np.float64)), _ptr(st.view(np.float64)))
    if rc:
        raise ValueError("ETD: k must be positive")
    return (out, st) if want_stage else out


# ---- drivers (plain loops over the steppers above) ------------------------
def run_fixed(m: Model, scheme: str, uh0, k: float, nsteps: int, r0=None, psd_tol=1e-10,
              psd_iters=None, record=False):
    """Fixed-step trajectory: a first-order startup step from u^0, then BDF2
    steps of size k (ETDRK2, a one-step method, takes nsteps equal steps).
    ``psd_iters`` (list) replays a per-step PSD iteration count.  Returns the
    final spectrum (and the list of states if record)."""
    un = _cplx(uh0)
    um = None
    r_n = r_nm1 = None
    if scheme == "sav":
        r_n = r0 if r0 is not None else float(np.sqrt(E1(m, un) + m.D0))
        r_nm1 = r_n
    states = [un] if record else None
    iters = []
    for n in range(nsteps):
        k_n = -1.0 if n == 0 else k
        if scheme == "imex":
            new = imex_step(m, un, um, k, k_n)
        elif scheme == "sav":
            new, r_new = sav_step(m, un, um, r_n, r_nm1, k, k_n)
            r_nm1, r_n = r_n, r_new
        elif scheme == "etd":  # one-step method: no startup step
            new = etd_step(m, un, k)
        elif scheme == "psd":
            fi = psd_iters[n] if psd_iters is not None else 0
            new, it, _, rc = psd_step(m, un, um, k, k_n, tol=psd_tol, fixed_iters=fi)
            iters.append(it)
        else:
            raise ValueError(scheme)
        um, un = un, new
        if record:
            states.append(un)
    if record:
        return un, states
    return un


# ---- learned warm start network (nn_oracle.c) ---------------------------------
def bf16(x):
    """Round to the nearest bfloat16 (ties to even), elementwise."""
    x = np.asarray(x, dtype=np.float64)
    f = x.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    special = (u & 0x7F800000) == 0x7F800000
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    r = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(special, x, r)


def nn_conv_fwd(x, w, bias, round_bf16=True):
    """x (B, H, W, 32), w (9, cout, 32), bias (cout,): (z, y) for cout 32, o for 16."""
    x, w, bias = _real(x), _real(w), _real(bias)
    B, H, W, _ = x.shape
    cout = w.shape[1]
    z = np.zeros((B, H, W, 32))
    y = np.zeros((B, H, W, 32))
    o = np.zeros((B, H, W))
    _load().nn_conv_fwd(B, H, W, cout, _ptr(x), _ptr(w), _ptr(bias), _ptr(z), _ptr(y), _ptr(o),
                        int(round_bf16))
    return (z, y) if cout == 32 else o


def nn_conv_bwd_data(dz, w, z_prev, round_bf16=True):
    dz, w, z_prev = _real(dz), _real(w), _real(z_prev)
    B, H, W, _ = dz.shape
    out = np.zeros((B, H, W, 32))
    _load().nn_conv_bwd_data(B, H, W, w.shape[1], _ptr(dz), _ptr(w), _ptr(z_prev), _ptr(out),
                             int(round_bf16))
    return out


def nn_conv_bwd_w(dz, x, cout):
    dz, x = _real(dz), _real(x)
    B, H, W, _ = dz.shape
    dw = np.zeros((9, cout, 32))
    db = np.zeros(cout)
    _load().nn_conv_bwd_w(B, H, W, cout, _ptr(dz), _ptr(x), _ptr(dw), _ptr(db))
    return dw, db


def nn_mse(o, t, round_bf16=True):
    o, t = _real(o), _real(t)
    dz = np.zeros(o.shape + (32,))
    loss = _load().nn_mse(o.size, _ptr(o), _ptr(t), _ptr(dz), int(round_bf16))
    return loss, dz


def nn_loss_and_grads(x, params, target, round_bf16=True):
    """Whole network: params = [(w, b), ...] (hidden layers cout 32, last
    cout 16).  Returns (loss, [(dw, db), ...], o)."""
    acts = [bf16(x) if round_bf16 else _real(x)]
    zs = []
    nl = len(params)
    for i, (w, b) in enumerate(params):
        wq = bf16(w) if round_bf16 else w
        if i < nl - 1:
            z, y = nn_conv_fwd(acts[-1], wq, b, round_bf16)
            zs.append(z)
            acts.append(y)
        else:
            o = nn_conv_fwd(acts[-1], wq, b, round_bf16)
    loss, dz = nn_mse(o, target, round_bf16)
    grads = [None] * nl
    for i in range(nl - 1, -1, -1):
        w, b = params[i]
        wq = bf16(w) if round_bf16 else w
        grads[i] = nn_conv_bwd_w(dz, acts[i], w.shape[1])
        if i > 0:
            dz = nn_conv_bwd_data(dz, wq, zs[i - 1], round_bf16)
    return loss, grads, o
