"""GPU test of fch_step_imex_static, the BDF2-IMEX step that allocates nothing
and keeps its intermediate spectra in the library's own device array.

It is called through the C ABI on plans that never received a workspace, and
checked bit for bit against fch_step_imex (same kernels, same launch
configuration) on two calls in a row, the second with a smaller grid, and
against the oracle's IMEX step to the one-step bound (1e-10 relative L2).
Sizes above the array's limit are refused before any device work."""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

from paper_2006_04784_amd import inputs

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_04784_amd import fch
    fch.lib()
    return fch


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def model_kw(N, L, eps=0.1):
    return dict(N=N, L=L, eps=eps, eta1=1.45, eta2=2.0, p=1, q=0.0, zeta=1.1, D0=L * L * 1.05)


def bare_plan(F, kw):
    """A plan made through the C ABI with no workspace set."""
    prm = F.fch_params(kw["N"], kw["L"], kw["eps"], kw["eta1"], kw["eta2"], kw["p"], kw["q"],
                       0.3, -1.0, 1.0, 2.0, 1.0, kw["zeta"], kw["D0"])
    h = C.c_void_p()
    assert F.lib().fch_plan_create(C.byref(prm), C.byref(h)) == F.FCH_OK
    F.lib().fch_plan_set_stream(h, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return h


def states(N, L, eps, seed):
    """(u^n, u^{n-1}) half spectra in the oracle's layout: a circle with noise
    and a slightly different copy of it."""
    import oracle
    u0 = inputs.circle_bilayer(N, L, eps, noise=1e-3, seed=seed)
    u1 = u0 + 1e-4 * inputs.white_noise(N, seed=seed + 1)
    return oracle.r2c(u1), oracle.r2c(u0)


def dev(uh_np):
    return torch.from_numpy(np.ascontiguousarray(uh_np.T)).to("cuda")


@pytest.mark.parametrize("sizes", [(512, 64), (256, 128)])
def test_static_step_equals_workspace_step(F, orc, sizes):
    k_np1, k_n = 1.3e-3, 1e-3
    for call, N in enumerate(sizes):
        L = N * 4 * np.pi / 256
        kw = model_kw(N, L)
        log("static IMEX step: call %d, N=%d" % (call, N))
        un, um = states(N, L, kw["eps"], seed=10 + N)
        d_un, d_um = dev(un), dev(um)
        ref_plan = F.Plan(**kw)
        ref = ref_plan.step_imex(d_un, d_um, k_np1, k_n)
        h = bare_plan(F, kw)
        try:
            out = torch.full_like(d_un, float("nan"))
            code = F.lib().fch_step_imex_static(h, C.c_void_p(d_un.data_ptr()),
                                                C.c_void_p(d_um.data_ptr()), k_np1, k_n,
                                                C.c_void_p(out.data_ptr()))
            assert code == F.FCH_OK, code
            torch.cuda.synchronize()
            # the same kernels on the same values: identical bits
            assert torch.equal(out, ref), float((out - ref).abs().max())
            # startup step (k_n <= 0, u^{n-1} not read)
            out0 = torch.full_like(d_un, float("nan"))
            assert F.lib().fch_step_imex_static(h, C.c_void_p(d_un.data_ptr()), None, k_np1,
                                                -1.0, C.c_void_p(out0.data_ptr())) == F.FCH_OK
            ref0 = ref_plan.step_imex(d_un, d_un, k_np1, -1.0)
            torch.cuda.synchronize()
            assert torch.equal(out0, ref0)
        finally:
            F.lib().fch_plan_destroy(h)
        m = orc.Model(**kw)
        e = rel(out.cpu().numpy().T, orc.imex_step(m, un, um, k_np1, k_n))
        log("  N=%d: bit-identical to fch_step_imex, oracle rel %.2e" % (N, e))
        assert e < 1e-10


def test_static_step_binding_and_limits(F, orc):
    N = 64
    kw = model_kw(N, 4 * np.pi)
    plan = F.Plan(**kw)
    un, um = states(N, kw["L"], kw["eps"], seed=3)
    d_un, d_um = dev(un), dev(um)
    a = plan.step_imex_static(d_un, d_um, 1e-3, 1e-3)
    b = plan.step_imex(d_un, d_um, 1e-3, 1e-3)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # u^{n+1} may alias u^{n-1}, as for fch_step_imex
    d_um2 = d_um.clone()
    plan.step_imex_static(d_un, d_um2, 1e-3, 1e-3, out=d_um2)
    torch.cuda.synchronize()
    assert torch.equal(d_um2, b)
    # beyond the scratch array's limit: refused, output untouched
    big = model_kw(2 * F.STATIC_MAX_N, 4 * np.pi)
    h = bare_plan(F, big)
    try:
        z = torch.zeros((big["N"] // 2 + 1, big["N"]), dtype=torch.complex128, device="cuda")
        o = torch.full_like(z, 7.0)
        code = F.lib().fch_step_imex_static(h, C.c_void_p(z.data_ptr()), C.c_void_p(z.data_ptr()),
                                            1e-3, 1e-3, C.c_void_p(o.data_ptr()))
        assert code == F.FCH_E_UNSUPPORTED
        torch.cuda.synchronize()
        assert bool((o == 7.0).all())
    finally:
        F.lib().fch_plan_destroy(h)
