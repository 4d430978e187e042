"""GPU tests of the learned warm start kernels: each BF16-MFMA convolution
kernel and a full training step against the FP64 oracle with bfloat16
rounding emulated at the same points (relative L2 per tensor)."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_04784_amd import fch
    fch.lib()
    return fch


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, float) - b) / max(np.linalg.norm(b), 1e-30))


def tb(a):   # exactly representable bf16 values -> torch bf16 on the GPU
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).cuda()


def tf(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def P(t):
    return C.c_void_p(t.data_ptr())


@pytest.mark.parametrize("B,H,W", [(2, 16, 32), (4, 128, 256)])
def test_conv_forward_both_launch_shapes(F, orc, B, H, W):
    """Forward convolutions under both workgroup shapes: 16 waves per tile for
    fewer than 512 tiles (inference sizes), 4 waves otherwise."""
    L = F.lib()
    rng = np.random.default_rng(5)
    x = orc.bf16(rng.normal(size=(B, H, W, 32)))
    w = orc.bf16(rng.normal(0, 0.1, size=(9, 32, 32)))
    bias = rng.normal(0, 0.1, size=32).astype(np.float32).astype(np.float64)
    z = torch.zeros((B, H, W, 32), dtype=torch.bfloat16, device="cuda")
    y = torch.zeros_like(z)
    y2 = torch.zeros_like(z)
    assert L.fch_nn_conv_fwd(B, H, W, 32, P(tb(x)), P(tb(w)), P(tf(bias)), P(z), P(y), None,
                             None) == 0
    assert L.fch_nn_conv_fwd(B, H, W, 32, P(tb(x)), P(tb(w)), P(tf(bias)), None, P(y2), None,
                             None) == 0
    zr, yr = orc.nn_conv_fwd(x, w, bias, True)
    assert rel(z.float().cpu().numpy(), zr) < 2e-3
    assert rel(y.float().cpu().numpy(), yr) < 2e-3
    assert torch.equal(y2, y)
    w16 = orc.bf16(rng.normal(0, 0.1, size=(9, 16, 32)))
    o = torch.zeros((B, H, W), dtype=torch.float32, device="cuda")
    assert L.fch_nn_conv_fwd(B, H, W, 16, P(tb(x)), P(tb(w16)), P(tf(bias[:16])), None, None,
                             P(o), None) == 0
    assert rel(o.cpu().numpy(), orc.nn_conv_fwd(x, w16, bias[:16], True)) < 1e-5


# (2, 16, 32): one column chunk in k_conv_bwd_w, 4 weight-gradient partials.
# (4, 64, 256): 8 chunks (interior chunk boundaries and their halos), 32
# partials, so every group of the two-stage reduction sums two.
@pytest.mark.parametrize("B,H,W", [(2, 16, 32), (4, 64, 256)])
def test_conv_kernels(F, orc, B, H, W):
    L = F.lib()
    rng = np.random.default_rng(3)
    errs = {}
    x = orc.bf16(rng.normal(size=(B, H, W, 32)))
    w = orc.bf16(rng.normal(0, 0.1, size=(9, 32, 32)))
    bias = rng.normal(0, 0.1, size=32).astype(np.float32).astype(np.float64)
    z = torch.zeros((B, H, W, 32), dtype=torch.bfloat16, device="cuda")
    y = torch.zeros_like(z)
    assert L.fch_nn_conv_fwd(B, H, W, 32, P(tb(x)), P(tb(w)), P(tf(bias)), P(z), P(y), None,
                             None) == 0
    zr, yr = orc.nn_conv_fwd(x, w, bias, True)
    errs["z"] = rel(z.float().cpu().numpy(), zr)
    errs["y"] = rel(y.float().cpu().numpy(), yr)
    # measured (2,16,32) / (4,64,256): z 1.0e-7 / 2.3e-5, y 7.8e-8 / 2.5e-5 (single
    # bf16 rounding flips where FP32 and FP64 sums straddle a rounding boundary)
    assert errs["z"] < 1e-4 and errs["y"] < 1e-4
    # inference form: no z, the same y bit for bit
    y2 = torch.zeros_like(y)
    assert L.fch_nn_conv_fwd(B, H, W, 32, P(tb(x)), P(tb(w)), P(tf(bias)), None, P(y2), None,
                             None) == 0
    assert torch.equal(y2, y)
    # output layer
    w16 = orc.bf16(rng.normal(0, 0.1, size=(9, 16, 32)))
    o = torch.zeros((B, H, W), dtype=torch.float32, device="cuda")
    assert L.fch_nn_conv_fwd(B, H, W, 16, P(tb(x)), P(tb(w16)), P(tf(bias[:16])), None, None,
                             P(o), None) == 0
    errs["o"] = rel(o.cpu().numpy(), orc.nn_conv_fwd(x, w16, bias[:16], True))
    assert errs["o"] < 1e-6   # measured 9.5e-8 (FP32 output, no bf16 rounding)
    # backward data, both weight shapes
    dz = orc.bf16(rng.normal(size=(B, H, W, 32)))
    zp = orc.bf16(rng.normal(size=(B, H, W, 32)))
    wt = torch.zeros(9 * 32 * 32, dtype=torch.bfloat16, device="cuda")
    for ww in (w, w16):
        dzz = dz.copy()
        if ww.shape[1] == 16:
            dzz[..., 16:] = 0.0
        out = torch.zeros((B, H, W, 32), dtype=torch.bfloat16, device="cuda")
        assert L.fch_nn_conv_bwd_data(B, H, W, ww.shape[1], P(tb(dzz)), P(tb(ww)), P(tb(zp)),
                                      P(out), P(wt), None) == 0
        errs["dz_prev/%d" % ww.shape[1]] = rel(out.float().cpu().numpy(),
                                               orc.nn_conv_bwd_data(dzz, ww, zp, True))
        assert errs["dz_prev/%d" % ww.shape[1]] < 1e-4   # measured <= 2.1e-5
    # backward weights
    for cout in (32, 16):
        dzz = dz.copy()
        dzz[..., cout:] = 0.0
        n = int(L.fch_nn_bwd_w_scratch_floats(B, H, W))
        scr = torch.zeros(n, dtype=torch.float32, device="cuda")
        g = torch.zeros(9 * cout * 32 + cout, dtype=torch.float32, device="cuda")
        assert L.fch_nn_conv_bwd_w(B, H, W, cout, P(tb(dzz)), P(tb(x)), P(g), P(scr), None) == 0
        dw, db = orc.nn_conv_bwd_w(dzz, x, cout)
        gg = g.cpu().numpy()
        errs["dw/%d" % cout] = rel(gg[:9 * cout * 32], dw.ravel())
        errs["db/%d" % cout] = rel(gg[9 * cout * 32:], db)
        # measured <= 2.9e-7 (FP32 accumulation of exact bf16 products)
        assert errs["dw/%d" % cout] < 2e-6 and errs["db/%d" % cout] < 2e-6
    print("conv kernels B=%d H=%d W=%d rel L2: %s" % (B, H, W, {k: "%.2e" % v for k, v in
                                                               errs.items()}), flush=True)


# (8, 64, 256): the 4-wave forward path (512 tiles), 8 column chunks and 64
# weight-gradient partials (four per reduction group), as in training.
@pytest.mark.parametrize("B,H,W", [(2, 16, 32), (8, 64, 256)])
def test_training_step_matches_oracle(F, orc, B, H, W):
    from paper_2006_04784_amd import nn
    rng = np.random.default_rng(4)
    net = nn.WarmStartNet(H, W, B, seed=5)
    params = net.init_params(5)
    params[-1] = (rng.normal(0, 0.05, size=(9, 16, 32)), rng.normal(0, 0.05, size=16))
    params[-1][0][:, 1:, :] = 0.0
    params[-1][1][1:] = 0.0
    net.set_params(params)
    un = torch.from_numpy(rng.normal(size=(B, H, W))).cuda()
    um = un + 0.01 * torch.from_numpy(rng.normal(size=(B, H, W))).cuda()
    up = un + 0.012 * torch.from_numpy(rng.normal(size=(B, H, W))).cuda()
    k = torch.tensor([[2e-3, 1e-3], [1e-3, 1e-3]] * (B // 2), dtype=torch.float64).cuda()
    net.features(un, um, k, up)
    x = net.x.float().cpu().numpy().astype(np.float64)
    t = net.target.cpu().numpy().astype(np.float64)
    # features against their definition
    d = (un - um).cpu().numpy() * (k[:, 0] / k[:, 1]).cpu().numpy()[:, None, None]
    s = np.sqrt((d ** 2).mean(axis=(1, 2)))
    assert np.allclose(net.scale.cpu().numpy(), s, rtol=1e-12)
    assert np.array_equal(x[..., 0], orc.bf16(un.cpu().numpy()))
    assert np.allclose(t, ((up - un).cpu().numpy() - d) / s[:, None, None], rtol=1e-6, atol=1e-6)
    net.forward(B)
    loss = float(net.backward(B).cpu()[0])
    q = [(orc.bf16(w), b.astype(np.float32).astype(np.float64)) for w, b in params]
    lref, gref, oref = orc.nn_loss_and_grads(x, q, t, True)
    e_o = rel(net.o.cpu().numpy(), oref)
    e_loss = abs(loss - lref) / lref
    e_g = [(rel(gw, rw), rel(gb, rb)) for (gw, gb), (rw, rb) in zip(net.get_grads(), gref)]
    print("training step B=%d H=%d W=%d: output %.2e, loss %.2e, (dw, db) per layer %s"
          % (B, H, W, e_o, e_loss, ["(%.2e, %.2e)" % g for g in e_g]), flush=True)
    # measured at (2,16,32) / (8,64,256): output 2.8e-5 / 3.7e-4, loss 3.8e-7 /
    # 2.3e-7, gradients per tensor at most 4.1e-4 / 9.2e-5 (the first layer's
    # weights, whose gradient collects the bf16 rounding flips of all later
    # layers); the bound is the per-tensor 1e-3 of the learned net's pin
    assert e_o < 1e-3
    assert e_loss < 1e-5
    for ew, eb in e_g:
        assert ew < 1e-3
        assert eb < 1e-3
    # Adam: the first bias-corrected step from zero moments is
    # lr * g / (|g| + eps) against the gradient
    before = net.P.clone()
    net.adam(lr=1e-3, eps=1e-8)
    delta = (net.P - before).cpu().numpy().astype(np.float64)
    g = net.G.cpu().numpy().astype(np.float64)
    want = -1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(delta, want, rtol=1e-3, atol=5e-7)
    assert np.all(delta[g == 0.0] == 0.0)


def test_learned_warm_start_gain(F):
    """Trained on PSD step pairs of the 256^2 three-bilayer workload, the
    network's guess needs fewer PSD iterations than the extrapolated guess on
    two held-out trajectories, by a margin on the mean, at the same stopping
    tolerance and to the same solution; the untrained network (zero output
    layer) is the extrapolation."""
    from paper_2006_04784_amd import learned, nn
    plan = F.Plan(**learned.c5_model())
    te = [learned.psd_trajectory(plan, learned.c5_initial(200), 25)]
    net0 = nn.WarmStartNet(256, 256, 8, seed=0)
    ev0 = learned.evaluate(plan, net0, te)
    assert all(r[0] == r[1] for r in ev0["per_step"])
    ev, net, _ = learned.run_experiment(range(10), [200, 201], nsteps=60, epochs=15, batch=8)
    print({k: v for k, v in ev.items() if k != "per_step"}, flush=True)
    assert ev["loss_last"] < 0.3 * ev["loss_first"]
    # at least half an iteration per step fewer on the mean over both trajectories
    assert ev["iters_learned"] <= ev["iters_plain"] - 0.5
    # and fewer FFT calls, counting the transform of the guess
    assert ev["fft_calls_per_step_learned"] < ev["fft_calls_per_step_plain"]
    assert ev["max_rel_diff_solutions"] < 1e-8


def test_stored_parameters_round_trip_and_evaluate(F, tmp_path):
    """save_params / load_params reproduce a trained network's parameters and
    guess bit for bit; the stored full-scale parameters drive the held-out
    comparison to the same solutions as the plain solver."""
    from paper_2006_04784_amd import learned, nn
    plan = F.Plan(**learned.c5_model())
    S, ks = learned.psd_trajectory(plan, learned.c5_initial(202), 6)
    net = nn.WarmStartNet(256, 256, 1, seed=0)
    net.load_params(learned.WEIGHTS_C5)
    path = str(tmp_path / "w")   # no suffix: written at exactly this path
    net.save_params(path)
    net2 = nn.WarmStartNet(256, 256, 1, seed=3)
    net2.load_params(path)
    assert torch.equal(net.P, net2.P) and torch.equal(net.PB, net2.PB)
    k = torch.tensor([[ks[3], ks[2]]], dtype=torch.float64, device="cuda")
    g1 = net.guess(S[2:3].contiguous(), S[1:2].contiguous(), k).clone()
    g2 = net2.guess(S[2:3].contiguous(), S[1:2].contiguous(), k)
    assert torch.equal(g1, g2)
    ev = learned.evaluate(plan, net, [(S, ks)])
    print({k_: v for k_, v in ev.items() if k_ != "per_step"}, flush=True)
    assert ev["steps"] == 5 and ev["max_rel_diff_solutions"] < 1e-8
    with pytest.raises(ValueError):   # another architecture's file
        nn.WarmStartNet(256, 256, 1).load_params(_bad_params(tmp_path))


def _bad_params(tmp_path):
    p = str(tmp_path / "bad.npz")
    with open(p, "wb") as fh:
        np.savez(fh, params=np.zeros(7, np.float32), layers=np.array([32]), ch=np.int64(32),
                 in_ch=np.int64(3))
    return p
