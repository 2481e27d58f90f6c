"""Pins of the learned-guess oracle (oracle/convnet.py), no GPU.

Each pin checks the oracle against something other than itself: torch's own
FP32 -> BF16 conversion, scipy's N-d correlation, the adjoint identities
that define the transposed convolution and the weight gradient, central
finite differences of the loss, closed forms of Adam and worked feature
values.  ``test_convnet_mutants`` plants plausible mistakes in the oracle
and requires a pin to catch each one.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import scipy.ndimage
import torch

import oracle
import oracle.convnet as cn
from paper_1910_06059_amd import cases
from paper_1910_06059_amd.cases import MD, PSI, STB, DAY, Well


def _rng(seed=0):
    return np.random.default_rng(seed)


# ------------------------------------------------------------------ pins
def pin_bf16_matches_torch():
    """Round to nearest even FP32 -> BF16, as torch converts."""
    rng = _rng(1)
    x = np.concatenate([
        rng.standard_normal(4000) * 10.0 ** rng.integers(-30, 30, 4000),
        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0, -0.0,
                  np.inf, -np.inf, 1e-40, 3.0e38, 2.0 ** -133]),
    ])
    ours = cn.to_bf16_bits(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).view(torch.int16)
    ref = ref.numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    nan = cn.from_bf16_bits(cn.to_bf16_bits(np.array([np.nan])))
    assert np.isnan(nan[0])
    # exact values survive, ties go to even
    assert cn.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert cn.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def pin_conv_matches_scipy_correlate():
    """conv is a zero-padded 3x3x3 cross-correlation summed over input
    channels: out[..., o] = b[o] + sum_i correlate(x[..., i], K[o, i])."""
    rng = _rng(2)
    nz, ny, nx = 4, 5, 6
    x = rng.standard_normal((nz, ny, nx, cn.CH))
    W = rng.standard_normal((cn.TAPS, cn.CH, cn.CH))
    b = rng.standard_normal(cn.CH)
    out = cn.conv(x, W, b)
    K = np.zeros((cn.CH, cn.CH, 3, 3, 3))    # [o][i][z][y][x]
    for t in range(cn.TAPS):
        dx, dy, dz = t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1
        K[:, :, dz + 1, dy + 1, dx + 1] = W[t]
    ref = np.zeros_like(out)
    for o in range(cn.CH):
        ref[..., o] = b[o]
        for i in range(cn.CH):
            ref[..., o] += scipy.ndimage.correlate(x[..., i], K[o, i], mode="constant", cval=0.0)
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-11)


def pin_conv_transpose_is_adjoint():
    """<conv(x, W), d> = <x, conv_transpose(d, W)>."""
    rng = _rng(3)
    x = rng.standard_normal((3, 4, 5, cn.CH))
    d = rng.standard_normal((3, 4, 5, cn.CH))
    W = rng.standard_normal((cn.TAPS, cn.CH, cn.CH))
    lhs = np.sum(cn.conv(x, W) * d)
    rhs = np.sum(x * cn.conv_transpose(d, W))
    assert abs(lhs - rhs) <= 1e-10 * np.sum(np.abs(cn.conv(np.abs(x), np.abs(W)) * np.abs(d)))


def pin_weight_grad_is_adjoint():
    """<conv(x, W, b), d> = <W, dW(x, d)> + <b, db(d)>."""
    rng = _rng(4)
    x = rng.standard_normal((2, 3, 7, cn.CH))
    d = rng.standard_normal((2, 3, 7, cn.CH))
    W = rng.standard_normal((cn.TAPS, cn.CH, cn.CH))
    b = rng.standard_normal(cn.CH)
    dW, db = cn.conv_weight_grad(x, d)
    lhs = np.sum(cn.conv(x, W, b) * d)
    rhs = np.sum(W * dW) + np.sum(b * db)
    assert abs(lhs - rhs) <= 1e-10 * np.sum(cn.conv_abs(x, W, b) * np.abs(d))


def _random_params(seed, scale=0.3):
    rng = _rng(seed)
    return rng.standard_normal(cn.PARAMS) * scale


def pin_network_gradient_matches_finite_differences():
    """backward() of the exact (unrounded) network is the derivative of the
    loss: central differences along random directions."""
    rng = _rng(5)
    shape = (3, 4, 5)
    n_box = 60
    cell_box = np.sort(rng.choice(n_box, 45, replace=False))
    feats = cn.to_box(rng.standard_normal((45, 11)), cell_box, shape)
    tgt = rng.standard_normal((45, 3)) * 0.3
    params = _random_params(6)

    def loss(p):
        _, out = cn.forward(feats, p, rounded=False)
        return cn.loss_and_dout(out, tgt, cell_box, rounded=False)[0]

    acts, out = cn.forward(feats, params, rounded=False)
    _, dout = cn.loss_and_dout(out, tgt, cell_box, rounded=False)
    g = cn.backward(acts, dout, params, rounded=False)
    for k in range(4):
        v = rng.standard_normal(cn.PARAMS)
        if k == 3:    # the last layer's bias alone
            v = np.zeros(cn.PARAMS)
            v[2 * cn.LAYER + cn.LAYER_W:] = rng.standard_normal(cn.CH)
        h = 1e-6
        fd = (loss(params + h * v) - loss(params - h * v)) / (2 * h)
        an = float(g @ v)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.linalg.norm(g) * np.linalg.norm(v)), (k, fd, an)


def pin_adam_closed_forms():
    """Adam: the first update is lr g / (|g| + eps); under a constant
    gradient the bias-corrected moments stay g and g^2, so every update is
    the same."""
    rng = _rng(7)
    g = rng.standard_normal(50)
    w0 = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    w, m, v = cn.adam(w0, g, np.zeros(50), np.zeros(50), 1, lr)
    assert np.allclose(w, w0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    for step in range(2, 6):
        w_prev = w
        w, m, v = cn.adam(w, g, m, v, step, lr)
        assert np.allclose(w_prev - w, lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-15)


def pin_loss_closed_form():
    """A constant error e in every output gives loss e^2 over the two
    saturation outputs and dL/dout = 2e/(2n) there, zero for the unused
    pressure output whatever its error; with cells left out the sum shrinks
    but the divisor stays 2n."""
    rng = _rng(8)
    shape = (2, 2, 3)
    cell_box = np.array([0, 2, 3, 5, 7, 11])
    tgt = rng.standard_normal((6, 3))
    e = 0.25
    o = tgt + e
    o[:, 0] += 7.0                      # the pressure output does not count
    out = cn.to_box(o, cell_box, shape)
    loss, d = cn.loss_and_dout(out, tgt, cell_box, rounded=False)
    assert abs(loss - e * e) <= 1e-15
    dd = d.reshape(-1, cn.CH)
    assert np.allclose(dd[cell_box, 1:3], 2 * e / 12.0, rtol=1e-15, atol=0)
    assert not np.any(dd[:, 0]) and not np.any(dd[:, 3:])
    assert not np.any(np.delete(dd, cell_box, axis=0))
    # cells outside `free` contribute nothing but the count stays n
    free = np.array([True, False, True, True, False, True])
    loss2, d2 = cn.loss_and_dout(out, tgt, cell_box, rounded=False, free=free)
    assert abs(loss2 - e * e * 4.0 / 6.0) <= 1e-15
    dd2 = d2.reshape(-1, cn.CH)
    assert not np.any(dd2[cell_box[~free]]) and np.allclose(dd2[cell_box[free], 1:3], 2 * e / 12.0)


def _feature_case():
    c = cases.box_case(2, 1, 1, dx=100.0, dy=100.0, dz=5.0, median_md=100.0, sigma_ln=0.0,
                       wells=[Well("I", cases.WELL_RATE_INJ, [(0, 0, 0)], 500 * STB / DAY,
                                   phase=cases.W),
                              Well("P", cases.WELL_BHP_PROD, [(1, 0, 0)], 3000.0 * PSI)])
    c.perm_h[:] = 100.0 * MD
    return c


def pin_features_worked_values():
    """Feature channels of a two-cell box with one water injector and one
    producer, written out by hand."""
    c = _feature_case()
    m = oracle.Model(c)
    cell, wi, well = m.conns()
    y_n = np.array([[5300.0 * PSI, 0.2, 0.05], [3400.0 * PSI, 0.3, 0.0]])
    y_nm1 = np.array([[4300.0 * PSI, 0.12, 0.0], [4800.0 * PSI, 0.12, 0.0]])
    f = cn.features(c, y_n, y_nm1, np.arange(2), cell, wi, well, rounded=False).reshape(2, cn.CH)
    assert abs(f[0, 0] - 0.5) < 1e-15 and abs(f[1, 0] + 1.4) < 1e-15
    assert abs(f[0, 3] - 10.0) < 1e-13 and abs(f[1, 3] + 14.0) < 1e-13
    assert np.array_equal(f[:, 1:3], y_n[:, 1:3])
    assert np.allclose(f[:, 4:6], [[0.8, 0.5], [1.8, 0.0]], rtol=1e-14, atol=0)
    assert np.allclose(f[:, 6], 0.0, atol=1e-15)          # 100 mD
    q = 500 * STB / DAY
    assert abs(f[0, 7] - q * 86400.0 / 10.0) <= 1e-12 * f[0, 7]
    assert f[1, 7] == 0.0 and not np.any(f[:, 8:10])
    wi_p = wi[list(well).index(1)]
    expect = math.log(1.0 + wi_p * (400.0 * PSI) / 1e-3 * 86400.0 / 10.0)
    assert abs(f[1, 10] - expect) <= 1e-14 * expect and f[0, 10] == 0.0
    # below the BHP the producer term vanishes
    y_low = y_n.copy()
    y_low[1, 0] = 2900.0 * PSI
    f2 = cn.features(c, y_low, y_nm1, np.arange(2), cell, wi, well, rounded=False).reshape(2, cn.CH)
    assert f2[1, 10] == 0.0
    assert not np.any(f[:, 11:])


def pin_apply_guess_special_cases():
    """The guess is y_n + (y_n - y_{n-1}) plus the saturation correction (ds
    per 0.1; the pressure output is ignored, the pressure is extrapolated);
    saturations clamped, s_g lowered to keep s_w + s_g <= 1, a non-finite
    output dropping the whole correction (the extrapolation remains)."""
    y_n = np.array([[1e7, 0.5, 0.2], [2e7, 0.1, 0.1], [3e7, 0.9, 0.05], [4e7, 0.3, 0.3]])
    y_nm1 = np.array([[1e7 - 50 * PSI, 0.45, 0.2], [2e7, 0.1, 0.1], [3e7, 0.8, 0.05],
                      [4e7 + 10 * PSI, 0.3, 0.35]])
    out = np.zeros((1, 1, 4, cn.CH))
    out[0, 0, 0, :3] = [1.0, 1.0, -0.5]
    out[0, 0, 1, :3] = [-2.0, -5.0, 15.0]
    out[0, 0, 2, :3] = [0.0, 2.0, 1.0]
    out[0, 0, 3, :3] = [np.nan, 1.0, 1.0]
    g = cn.apply_guess(y_n, y_nm1, out, np.arange(4))
    assert np.allclose(g[0], [1e7 + 50 * PSI, 0.65, 0.15], rtol=1e-15, atol=1e-15)
    assert np.allclose(g[1], [2e7, 0.0, 1.0], rtol=1e-15)
    assert np.allclose(g[2], [3e7, 1.0, 0.0], rtol=1e-15)
    assert np.allclose(g[3], [4e7 - 10 * PSI, 0.3, 0.25], rtol=1e-15, atol=1e-15)
    # cells outside `free` (well cells) keep the extrapolation
    free = np.array([False, True, True, True])
    g2 = cn.apply_guess(y_n, y_nm1, out, np.arange(4), free)
    assert np.allclose(g2[0], [1e7 + 50 * PSI, 0.55, 0.2], rtol=1e-15, atol=1e-15)
    assert np.array_equal(g2[1:], g[1:])
    # away from wells: no non-zero well channel in the 3x3x3 neighbourhood
    fb = np.zeros((1, 3, 5, cn.CH))
    fb[0, 1, 0, 10] = 0.5          # producer term at box (x=0, y=1)
    fb[0, 0, 4, 8] = -0.0          # a negative zero is zero
    cbox = np.arange(15)
    away = cn.away_from_wells(fb, cbox).reshape(3, 5)
    assert np.array_equal(away, [[False, False, True, True, True]] * 3)


def pin_targets_round_trip():
    """Targets vanish on a linear trajectory, and feeding the targets back as
    the correction reproduces y_next wherever no clamp acts."""
    rng = _rng(10)
    n = 40
    y_n = np.stack([4e7 + rng.uniform(-1e6, 1e6, n), rng.uniform(0.2, 0.4, n),
                    rng.uniform(0.05, 0.2, n)], axis=1)
    step = np.stack([rng.uniform(-2e5, 2e5, n), rng.uniform(-0.02, 0.02, n),
                     rng.uniform(-0.02, 0.02, n)], axis=1)
    assert np.allclose(cn.targets(y_n, y_n - step, y_n + step), 0.0, atol=1e-9)
    y_next = y_n + step + np.stack([rng.uniform(-3e4, 3e4, n), rng.uniform(-0.01, 0.01, n),
                                    rng.uniform(-0.01, 0.01, n)], axis=1)
    y_nm1 = y_n - step
    t = cn.targets(y_n, y_nm1, y_next)
    out = cn.to_box(t, np.arange(n), (1, 1, n))
    got = cn.apply_guess(y_n, y_nm1, out, np.arange(n))
    assert np.allclose(got[:, 1:], y_next[:, 1:], rtol=1e-12, atol=1e-12)
    assert np.array_equal(got[:, 0], y_n[:, 0] + (y_n[:, 0] - y_nm1[:, 0]))


def pin_forward_identity_network():
    """Centre-tap identity weights pass the (ReLU'd, BF16) input through:
    a closed form of the whole forward pass."""
    rng = _rng(9)
    feats = np.abs(rng.standard_normal((3, 3, 4, cn.CH)))
    p = np.zeros(cn.PARAMS)
    for l in range(3):
        W = np.zeros((cn.TAPS, cn.CH, cn.CH))
        W[13] = np.eye(cn.CH)
        p[l * cn.LAYER:l * cn.LAYER + cn.LAYER_W] = W.ravel()
    acts, out = cn.forward(feats, p, rounded=True)
    assert np.array_equal(out, cn.bf16(feats))
    # one-cell shift: tap (dx=+1) moves data by one cell in -x
    p2 = np.zeros(cn.PARAMS)
    W = np.zeros((cn.TAPS, cn.CH, cn.CH))
    W[14] = np.eye(cn.CH)
    p2[2 * cn.LAYER:2 * cn.LAYER + cn.LAYER_W] = W.ravel()
    h = cn.conv(feats, W)
    assert np.array_equal(h[:, :, :-1], feats[:, :, 1:]) and not np.any(h[:, :, -1])


ALL_PINS = [pin_bf16_matches_torch, pin_conv_matches_scipy_correlate,
            pin_conv_transpose_is_adjoint, pin_weight_grad_is_adjoint,
            pin_network_gradient_matches_finite_differences, pin_adam_closed_forms,
            pin_loss_closed_form, pin_features_worked_values, pin_apply_guess_special_cases,
            pin_targets_round_trip, pin_forward_identity_network]


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_pin(pin):
    pin()


# --------------------------------------------------------------- mutants
def _mut_tap_swap(t):
    return (t // 3) % 3 - 1, t % 3 - 1, t // 9 - 1


def _mut_transpose_noflip(d, W):
    out = np.zeros(d.shape[:3] + (W.shape[2],))
    for t in range(cn.TAPS):
        out += cn._shifted(d, *cn.tap_offset(t)) @ W[t]
    return out


_orig_wgrad = cn.conv_weight_grad


def _mut_wgrad_transposed(x, d):
    dW, db = _orig_wgrad(x, d)
    return np.transpose(dW, (0, 2, 1)).copy(), db


def _mut_bf16_truncate(x):
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def _mut_adam_no_correction(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    return w - lr * m / (np.sqrt(v) + eps), m, v


def _mut_backward_nomask(acts, dout, params, rounded=True):
    r = cn.bf16 if rounded else (lambda v: np.asarray(v, dtype=np.float64))
    layers = cn.split(params)
    grad = np.zeros(cn.PARAMS)
    d = dout
    for l in (2, 1, 0):
        dW, db = cn.conv_weight_grad(acts[l], d)
        grad[l * cn.LAYER:l * cn.LAYER + cn.LAYER_W] = dW.ravel()
        grad[l * cn.LAYER + cn.LAYER_W:(l + 1) * cn.LAYER] = db
        if l > 0:
            d = r(cn.conv_transpose(d, r(layers[l][0])))
    return grad


_orig_loss = cn.loss_and_dout


def _mut_loss_over_n(out, tgt, cell_box, rounded=True):
    loss, d = _orig_loss(out, tgt, cell_box, rounded)
    return loss * 3.0, d


_orig_apply = cn.apply_guess


def _mut_apply_noclamp(y_n, y_nm1, out, cell_box):
    o = out.reshape(-1, out.shape[3])[np.asarray(cell_box), :3]
    e = 2 * np.asarray(y_n) - np.asarray(y_nm1)
    return e + np.stack([0.0 * o[:, 0], cn.DSS * o[:, 1], cn.DSS * o[:, 2]], axis=1)


def _mut_apply_pressure_corrected(y_n, y_nm1, out, cell_box):
    g = _orig_apply(y_n, y_nm1, out, cell_box)
    o = out.reshape(-1, out.shape[3])[np.asarray(cell_box), 0]
    g[:, 0] += cn.DPS * np.where(np.isfinite(o), o, 0.0)
    return g


def _mut_loss_trains_pressure(out, tgt, cell_box, rounded=True, free=None):
    loss, d = _orig_loss(out, tgt, cell_box, rounded, free)
    o = out.reshape(-1, out.shape[3])[np.asarray(cell_box), 0]
    dd = d.reshape(-1, d.shape[3]).copy()
    dd[np.asarray(cell_box), 0] = 2.0 * (o - tgt[:, 0]) / (2.0 * tgt.shape[0])
    return loss, dd.reshape(d.shape)


def _mut_apply_noskip(y_n, y_nm1, out, cell_box):
    return _orig_apply(y_n, y_n, out, cell_box)


def _mut_targets_noskip(y_n, y_nm1, y_next):
    return _orig_targets(y_n, y_n, y_next)


_orig_targets = cn.targets


MUTANTS = {
    "tap_offset_xy_swapped": ("tap_offset", _mut_tap_swap),
    "transpose_without_flip": ("conv_transpose", _mut_transpose_noflip),
    "weight_grad_transposed": ("conv_weight_grad", _mut_wgrad_transposed),
    "bf16_truncates": ("to_bf16_bits", _mut_bf16_truncate),
    "adam_without_bias_correction": ("adam", _mut_adam_no_correction),
    "backward_without_relu_mask": ("backward", _mut_backward_nomask),
    "loss_mean_over_n": ("loss_and_dout", _mut_loss_over_n),
    "guess_without_clamp": ("apply_guess", _mut_apply_noclamp),
    "guess_corrects_pressure": ("apply_guess", _mut_apply_pressure_corrected),
    "loss_trains_pressure": ("loss_and_dout", _mut_loss_trains_pressure),
    "guess_without_skip": ("apply_guess", _mut_apply_noskip),
    "targets_without_skip": ("targets", _mut_targets_noskip),
    "saturation_scale": ("DSS", 1.0),
    "pressure_offset": ("P0", 4700.0 * PSI),
    "injection_scale": ("QS", 86400.0),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_convnet_mutants(name, monkeypatch):
    attr, repl = MUTANTS[name]
    monkeypatch.setattr(cn, attr, repl)
    caught = []
    for pin in ALL_PINS:
        try:
            pin()
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"
