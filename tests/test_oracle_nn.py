"""Pins of the oracle's warm-start network: bfloat16 rounding against
hand-worked values, and the backward pass against central finite
differences of the FP64 loss (no rounding)."""
import numpy as np
import pytest


def test_bf16_rounding(orc):
    one = 1.0
    ulp = 2.0 ** -7                     # bfloat16 spacing at 1
    cases = [(one, one), (one + ulp / 2, one), (one + 3 * ulp / 2, one + 2 * ulp),
             (one + ulp / 2 + 2 ** -20, one + ulp), (-(one + 3 * ulp / 2), -(one + 2 * ulp)),
             (0.0, 0.0), (3.0, 3.0), (1e-3, 0.00099945068359375)]
    for x, want in cases:
        assert orc.bf16(x) == want, x
        assert orc._load().nn_bf16(x) == want, x


def _tiny(rng, B=1, H=4, W=6):
    x = np.zeros((B, H, W, 32))
    x[..., :3] = rng.normal(size=(B, H, W, 3))
    params = []
    for i, cout in enumerate((32, 32, 16)):
        w = rng.normal(0, 0.3, size=(9, cout, 32))
        if i == 0:
            w[:, :, 3:] = 0.0
        params.append((w, rng.normal(0, 0.1, size=cout)))
    t = rng.normal(size=(B, H, W))
    return x, params, t


def test_backward_matches_finite_differences(orc):
    rng = np.random.default_rng(0)
    x, params, t = _tiny(rng)
    loss, grads, _ = orc.nn_loss_and_grads(x, params, t, round_bf16=False)
    h = 1e-6
    for li, (w, b) in enumerate(params):
        idx = [(rng.integers(9), rng.integers(w.shape[1] if li < 2 else 1),
                rng.integers(3 if li == 0 else 32)) for _ in range(4)]
        for (tp, co, ci) in idx:
            wp = [(ww.copy(), bb.copy()) for ww, bb in params]
            wm = [(ww.copy(), bb.copy()) for ww, bb in params]
            wp[li][0][tp, co, ci] += h
            wm[li][0][tp, co, ci] -= h
            fp = orc.nn_loss_and_grads(x, wp, t, round_bf16=False)[0]
            fm = orc.nn_loss_and_grads(x, wm, t, round_bf16=False)[0]
            fd = (fp - fm) / (2 * h)
            g = grads[li][0][tp, co, ci]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (li, tp, co, ci, fd, g)
        co = 0
        bp = [(ww.copy(), bb.copy()) for ww, bb in params]
        bm = [(ww.copy(), bb.copy()) for ww, bb in params]
        bp[li][1][co] += h
        bm[li][1][co] -= h
        fd = (orc.nn_loss_and_grads(x, bp, t, False)[0] - orc.nn_loss_and_grads(x, bm, t, False)[0]) / (2 * h)
        assert abs(fd - grads[li][1][co]) <= 1e-6 * max(1.0, abs(fd))


def test_conv_periodic_shift_identity(orc):
    """A single tap of weight 1 shifts the field periodically."""
    rng = np.random.default_rng(1)
    x = np.zeros((1, 4, 6, 32))
    x[..., 0] = rng.normal(size=(4, 6))
    w = np.zeros((9, 16, 32))
    w[2, 0, 0] = 1.0                    # tap (dy, dx) = (-1, +1)
    o = orc.nn_conv_fwd(x, w, np.zeros(16), round_bf16=False)
    assert np.allclose(o[0], np.roll(np.roll(x[0, :, :, 0], 1, axis=0), -1, axis=1))
