"""GPU: the one-launch PSD solve (Sec. 3.3) -- every iteration of a solve in
one persistent kernel with device-wide barriers and the stopping test on the
device -- against the oracle at the GPU's iteration count, against the
separate row and column launches of the same variant pair (the same
arithmetic, contracted differently by the compiler: equal to rounding),
under graph capture, and its launch count."""
import sys

import numpy as np
import pytest
import torch

from paper_2006_04784_amd import inputs

pytestmark = pytest.mark.gpu

# the row / column variant pair each one-launch solve is compiled with
PAIR = {256: (2, 8, 0, 4, 0), 512: (2, 8, 0, 4, 0), 1024: (2, 8, 0, 4, 0),
        2048: (2, 16, 0, 8, 0)}


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


def dev(uh_np):
    return torch.from_numpy(np.ascontiguousarray(uh_np.T)).to("cuda")


def host(uh_t):
    return uh_t.cpu().numpy().T


def setup(F, orc, N, eps=0.1, k=1e-3):
    L = N * 4 * np.pi / 256
    kw = dict(N=N, L=L, eps=eps, eta1=1.45, eta2=2.0, p=1, q=0.0, zeta=1.1, D0=L * L * 1.05)
    plan, m = F.Plan(**kw), orc.Model(**kw)
    uh0 = orc.r2c(inputs.circle_bilayer(N, L, eps, seed=7, noise=1e-3))
    u1 = orc.imex_step(m, uh0, None, k, -1.0)
    return plan, m, uh0, u1


@pytest.mark.parametrize("N", [256, 512, 1024, 2048])
def test_one_launch_equals_separate_launches(F, orc, N):
    """The one-launch solve matches the oracle replaying its iteration count,
    stops where the separate launches of the same variant pair stop (within
    one iteration: the ratio near i_tol differs at rounding level), equals
    them to rounding at equal counts, and reaches max_iter with NOCONV."""
    log("one-launch PSD N=%d" % N)
    k = 1e-3 if N < 2048 else 1e-4
    plan, m, uh0, u1 = setup(F, orc, N, k=k)
    assert plan.get_psd_solve()[0] is False     # off by default
    plan.set_psd_solve(True)
    on, grid = plan.get_psd_solve()
    assert on and grid > 0
    plan.set_config(PAIR[N])
    a, b = dev(u1), dev(uh0)
    opts = dict(tol=1e-10) if N < 2048 else dict(fixed_iters=3)
    x1, s1 = plan.step_psd(a, b, 1.3 * k, k, **opts)
    plan.set_psd_solve(False)
    x0, s0 = plan.step_psd(a, b, 1.3 * k, k, **opts)
    plan.set_psd_solve(True)
    ref, _, _, _ = orc.psd_step(m, u1, uh0, 1.3 * k, k, fixed_iters=s1["iters"])
    e_orc, e_sep = rel(host(x1), ref), rel(host(x1), host(x0))
    log("  grid %d, %d / %d iterations (one launch / separate), vs oracle %.2e, vs separate "
        "%.2e" % (grid, s1["iters"], s0["iters"], e_orc, e_sep))
    assert e_orc < 1e-10
    assert abs(s1["iters"] - s0["iters"]) <= 1
    if s1["iters"] == s0["iters"]:
        assert e_sep < 1e-12
    # a fixed count and max_iter
    x1, s1 = plan.step_psd(a, b, 1.3 * k, k, fixed_iters=5)
    plan.set_psd_solve(False)
    x0, s0 = plan.step_psd(a, b, 1.3 * k, k, fixed_iters=5)
    plan.set_psd_solve(True)
    assert s1["iters"] == s0["iters"] == 5 and rel(host(x1), host(x0)) < 1e-12
    x1, s1 = plan.step_psd(a, b, 1.3 * k, k, tol=1e-30, max_iter=4, raise_noconv=False)
    assert s1["status"] == F.FCH_E_NOCONV and s1["iters"] == 4


def test_one_launch_is_one_launch(F, orc):
    """A converged 1024^2 solve: the initial-iterate column pass and one
    solve kernel, against two launches per iteration plus one."""
    plan, m, uh0, u1 = setup(F, orc, 1024)
    plan.set_psd_solve(True)
    a, b = dev(u1), dev(uh0)
    plan.reset_stats()
    _, st = plan.step_psd(a, b, 1e-3, 1e-3, tol=1e-10)
    one = plan.stats()["launches"]
    plan.set_psd_solve(False)
    plan.reset_stats()
    plan.step_psd(a, b, 1e-3, 1e-3, tol=1e-10)
    sep = plan.stats()["launches"]
    plan.set_psd_solve(True)
    log("  launches: one-launch %d, separate %d (%d iterations)" % (one, sep, st["iters"]))
    assert one <= 3 and sep >= 2 * st["iters"]


def test_one_launch_under_graph_capture(F, orc):
    """fch_step_psd_dev captured once and replayed with new step sizes and
    states written between replays: each replay equals the eager solve bit
    for bit, with the same iteration count, though the counts differ from
    replay to replay (the captured sequence does not depend on them)."""
    log("one-launch PSD under graph capture, 512^2")
    plan, m, uh0, u1 = setup(F, orc, 512)
    plan.set_psd_solve(True, grid=64)   # fewer workgroups than tasks: each loops
    k = 1e-3
    a0, a1 = dev(uh0), dev(u1)
    x_n, x_nm1, y = a1.clone(), a0.clone(), plan.spec()
    kd = torch.tensor([k, k], dtype=torch.float64, device="cuda")
    it = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.step_psd_dev(x_n, x_nm1, kd, y, it, st, tol=1e-10, max_iter=500)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.step_psd_dev(x_n, x_nm1, kd, y, it, st, tol=1e-10, max_iter=500)
    u2, _ = plan.step_psd(a1, a0, 2.0 * k, k, tol=1e-10)
    counts = set()
    for rep, (un, um, k1, k0) in enumerate([(a1, a0, 1.5 * k, k), (u2, a1, 4.0 * k, 2.0 * k),
                                            (a1, a0, 0.5 * k, k)]):
        x_n.copy_(un)
        x_nm1.copy_(um)
        kd.copy_(torch.tensor([k1, k0], dtype=torch.float64))
        g.replay()
        torch.cuda.synchronize()
        ref, s = plan.step_psd(un, um, k1, k0, tol=1e-10, max_iter=500)
        assert torch.equal(y, ref), rep
        assert int(it.item()) == s["iters"] and int(st.item()) == 0, rep
        counts.add(s["iters"])
    log("  iteration counts of the replays: %s" % sorted(counts))
    assert len(counts) > 1
