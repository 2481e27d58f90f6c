"""Learned Newton initial guess on the GPU (through the C ABI) against the
numpy oracle (oracle/convnet.py) and the CPU simulator oracle.

Tolerances follow from the arithmetic: the kernels multiply BF16 operands
exactly and add in FP32, so a layer output before rounding differs from the
FP64 sum by at most about n 2^-24 S (S the sum of |terms|, n <= 432 terms per
output, or the cell count for weight gradients); storing in BF16 adds at most
2^-9 relative on each side.  Bounds below use 1e-4 S (forward, transposed)
and 2e-4 S (weight gradient) plus 2^-8 relative for a BF16 result.
Whole-network comparisons allow for an occasional one-ulp BF16 flip of an
intermediate activation (when the FP32 and FP64 sums fall on either side of
a rounding boundary), so they use a bound relative to the output scale.
Converged states with the guess must match the oracle simulator to the path's
bar (1e-6 relative pressure, 1e-6 absolute saturations).
"""
import numpy as np
import pytest
import torch

import oracle
import oracle.convnet as cn
from paper_1910_06059_amd import cases
from paper_1910_06059_amd.cases import DAY, PSI, STB, Well

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def opm():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1910_06059_amd import opm as _opm
    _opm.init()
    return _opm


def _bits_to_dev(x):
    """float32 box [nz, ny, nx, 16] (BF16-exact) -> padded int16 rows on the GPU."""
    nz, ny, nx = x.shape[:3]
    rows = (nx * ny * nz + 15) // 16 * 16
    b = np.zeros((rows, cn.CH), dtype=np.uint16)
    b[:nx * ny * nz] = cn.to_bf16_bits(x.reshape(-1, cn.CH))
    return torch.from_numpy(b.view(np.int16)).cuda()


def _dev_to_box(t, shape, bf16=True):
    nz, ny, nx = shape
    a = t.cpu().numpy()[:nx * ny * nz]
    v = cn.from_bf16_bits(a.view(np.uint16)) if bf16 else a.astype(np.float64)
    return v.reshape(nz, ny, nx, cn.CH)


SHAPES = [(7, 11, 13), (1, 1, 1), (3, 2, 2), (2, 9, 33)]


def _params(seed):
    return cases.guess_init_params(seed, last_scale=1.0)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_pack_weights(opm, shape):
    p = _params(1)
    net = opm.GuessNet(p)
    wb = net.wbf16.cpu().numpy().view(np.uint16)
    for l, (W, _) in enumerate(cn.split(p)):
        fwd = wb[l * cn.LAYER_W:(l + 1) * cn.LAYER_W].reshape(cn.TAPS, cn.CH, cn.CH)
        bwd = wb[(3 + l) * cn.LAYER_W:(4 + l) * cn.LAYER_W].reshape(cn.TAPS, cn.CH, cn.CH)
        ref = cn.to_bf16_bits(W)
        assert np.array_equal(fwd, ref)
        assert np.array_equal(bwd, np.transpose(ref, (0, 2, 1)))


@pytest.mark.parametrize("relu", [True, False])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_conv_forward_parity(opm, shape, relu):
    x = cases.guess_random_feats(shape, seed=11, channels=16)
    p = _params(2)
    net = opm.GuessNet(p)
    for l in range(3):
        W, b = cn.split(p)[l]
        out = opm.guess_conv(shape, _bits_to_dev(x), net.w_fwd(l), net.bias(l), relu)
        torch.cuda.synchronize()
        got = _dev_to_box(out, shape, bf16=relu)
        Wr = cn.bf16(W)
        z = cn.conv(x.astype(np.float64), Wr, b)
        S = cn.conv_abs(x.astype(np.float64), Wr, b)
        ref = np.maximum(z, 0.0) if relu else z
        tol = 1e-4 * S + (2.0 ** -8 * np.abs(ref) if relu else 0.0)
        bad = np.abs(got - ref) > tol
        assert not bad.any(), (l, np.argwhere(bad)[:5], got[bad][:5], ref[bad][:5])
        # padding rows past the box are never written
        rows = out.cpu().numpy()[np.prod(shape):]
        assert not np.any(rows)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_conv_backward_parity(opm, shape):
    x = np.maximum(cases.guess_random_feats(shape, seed=12, channels=16), 0.0)
    d = cases.guess_random_feats(shape, seed=13, channels=16) * np.float32(1e-3)
    d = cn.bf16(d).astype(np.float32)
    p = _params(3)
    net = opm.GuessNet(p)
    for l in (1, 2):
        W, _ = cn.split(p)[l]
        Wr = cn.bf16(W)
        grad, din = opm.guess_conv_backward(shape, _bits_to_dev(x), _bits_to_dev(d),
                                            net.w_bwd(l), _bits_to_dev(x))
        torch.cuda.synchronize()
        x64, d64 = x.astype(np.float64), d.astype(np.float64)
        dW, db = cn.conv_weight_grad(x64, d64)
        SW, Sb = cn.conv_weight_grad(np.abs(x64), np.abs(d64))
        g = grad.cpu().numpy().astype(np.float64)
        ref = np.concatenate([dW.ravel(), db])
        S = np.concatenate([SW.ravel(), Sb])
        assert np.all(np.abs(g - ref) <= 2e-4 * S + 1e-30), np.max(np.abs(g - ref) / (S + 1e-30))
        gi = _dev_to_box(din, shape)
        zt = cn.conv_transpose(d64, Wr)
        St = cn.conv_transpose(np.abs(d64), np.abs(Wr))
        ref_i = np.where(x64 > 0, zt, 0.0)
        tol = 1e-4 * St + 2.0 ** -8 * np.abs(ref_i)
        assert np.all(np.abs(gi - ref_i) <= tol + 1e-30)
    # first layer: no input gradient requested
    grad, din = opm.guess_conv_backward(shape, _bits_to_dev(x), _bits_to_dev(d))
    assert din is None


def _guess_case():
    return cases.box_case(12, 10, 4, seed=21, dx=200 * cases.FT, dy=200 * cases.FT,
                          wells=[Well("I", cases.WELL_RATE_INJ, [(1, 1, k) for k in range(4)],
                                      1500 * STB / DAY),
                                 Well("G", cases.WELL_RATE_INJ, [(10, 1, 0)],
                                      2e3 * cases.MSCF / DAY, phase=cases.GAS),
                                 Well("P", cases.WELL_BHP_PROD, [(10, 8, 3)], 3000 * PSI),
                                 Well("P2", cases.WELL_BHP_PROD, [(2, 8, 0), (2, 8, 1)],
                                      3500 * PSI)],
                          report_dt=[10 * DAY] * 4, name="guess_box")


def _masked_guess_case():
    c = cases.box_case(9, 7, 4, seed=5, mask=cases.masked_mask(np.random.default_rng(8),
                                                                (4, 7, 9), 150), wells=[])
    act = np.argwhere(c.mask)
    k, j, i = act[0]
    k2, j2, i2 = act[-1]
    c.wells = [Well("I", cases.WELL_RATE_INJ, [(int(i), int(j), int(k))], 300 * STB / DAY),
               Well("P", cases.WELL_BHP_PROD, [(int(i2), int(j2), int(k2))], 3000 * PSI)]
    return c


FEATURE_CASES = {"box": _guess_case, "masked": _masked_guess_case, "C1": cases.config1}


def _oracle_feats(case, y_n, y_nm1, with_free=False):
    m = oracle.Model(case)
    cell, wi, well = m.conns()
    cb = m.geometry()["cell_box"]
    f = cn.features(case, y_n, y_nm1, cb, cell, wi, well)
    if with_free:
        return f, cb, cn.away_from_wells(f, cb)
    return f, cb


@pytest.mark.parametrize("name", list(FEATURE_CASES))
def test_features_parity(opm, name):
    case = FEATURE_CASES[name]()
    g = opm.GpuModel(case)
    y_n = cases.random_state(case, seed=3, p_jitter=1500 * PSI)
    y_nm1 = cases.random_state(case, seed=4)
    net = opm.GuessNet(_params(4))
    f = g.guess_features(net, g.state(y_n), g.state(y_nm1))
    got = _dev_to_box(f, (case.nz, case.ny, case.nx))
    ref, _ = _oracle_feats(case, y_n, y_nm1)
    # both sides round FP64 -> FP32 -> BF16; libm differences may move one ulp
    diff = np.abs(got - ref)
    assert np.all(diff <= 2.0 ** -7 * np.abs(ref))
    assert np.mean(got == ref) > 0.999
    rows = f.cpu().numpy()[case.n_box:]
    assert not np.any(rows)


@pytest.mark.parametrize("name", list(FEATURE_CASES))
def test_infer_parity(opm, name):
    case = FEATURE_CASES[name]()
    g = opm.GpuModel(case)
    y_n = cases.random_state(case, seed=5, p_jitter=800 * PSI)
    y_nm1 = cases.random_state(case, seed=6)
    p = _params(5)
    net = opm.GuessNet(p)
    yg = g.guess_infer(net, g.state(y_n), g.state(y_nm1)).cpu().numpy()
    feats, cb, free = _oracle_feats(case, y_n, y_nm1, with_free=True)
    _, out = cn.forward(feats, p)
    ref = cn.apply_guess(y_n, y_nm1, out, cb, free)
    o = out.reshape(-1, cn.CH)[cb, :3]
    scale = np.abs(o).max(axis=0)
    assert np.all(np.abs(yg[:, 0] - ref[:, 0]) <= 0.02 * cn.DPS * scale[0])
    for k in (1, 2):
        assert np.all(np.abs(yg[:, k] - ref[:, k]) <= 0.02 * scale[k] + 1e-15)
    assert np.all(yg[:, 1:] >= 0) and np.all(yg[:, 1:] <= 1)
    assert np.all(yg[:, 1] + yg[:, 2] <= 1.0 + 1e-15)


def test_train_step_parity(opm):
    case = _guess_case()
    g = opm.GpuModel(case)
    y_n = cases.random_state(case, seed=7, p_jitter=500 * PSI)
    y_nm1 = cases.random_state(case, seed=8)
    y_next = cases.random_state(case, seed=9, p_jitter=500 * PSI)
    p = _params(6)
    net = opm.GuessNet(p)
    lr = 1e-3
    loss = g.guess_train_step(net, g.state(y_n), g.state(y_nm1), g.state(y_next), lr)
    gl = float(loss.cpu()[0])
    w_gpu = net.params().astype(np.float64)
    feats, cb, free = _oracle_feats(case, y_n, y_nm1, with_free=True)
    acts, out = cn.forward(feats, p)
    tgt = cn.targets(y_n, y_nm1, y_next)
    rl, dout = cn.loss_and_dout(out, tgt, cb, free=free)
    grad = cn.backward(acts, dout, p)
    w_ref, _, _ = cn.adam(p.astype(np.float64), grad, 0.0, 0.0, 1, lr)
    assert abs(gl - rl) <= 2e-2 * rl
    # step 1 of Adam moves every parameter by about lr sign(g); compare where
    # the gradient is not small (a tiny gradient's sign is not determined)
    for l in range(3):
        sl = slice(l * cn.LAYER, (l + 1) * cn.LAYER)
        gg = grad[sl]
        big = np.abs(gg) > 0.05 * np.abs(gg).max()
        assert big.sum() > 10
        dw_gpu = (w_gpu - p)[sl][big]
        dw_ref = (w_ref - p)[sl][big]
        assert np.all(np.abs(dw_gpu - dw_ref) <= 0.02 * lr + 2e-7 * np.abs(p[sl][big])), l
    # training lowers the loss on a fixed sample
    losses = [gl]
    for _ in range(30):
        losses.append(float(g.guess_train_step(net, g.state(y_n), g.state(y_nm1),
                                               g.state(y_next), lr).cpu()[0]))
    assert losses[-1] < 0.7 * losses[0]


def test_select_parity(opm):
    case = _guess_case()
    g = opm.GpuModel(case)
    m = oracle.Model(case)
    dt = case.report_dt[0]
    y0 = case.initial_state()
    st, y1, _ = m.advance(y0.copy(), dt)
    assert st == 0
    acc0 = m.accumulation(y0)

    def max_cnv(y):
        _, R, _ = m.assemble(y, acc0, dt, jacobian=False)
        return np.max(m.norms(y, R, dt)[0])

    c_prev, c_good = max_cnv(y0), max_cnv(y1)
    yd = g.zeros_state()
    chosen, cnv = g.guess_select(yd, g.state(y0), g.state(y1), dt)
    assert chosen == 1
    assert abs(cnv[0] - c_prev) <= 1e-9 * c_prev and abs(cnv[1] - c_good) <= 1e-9 * c_good + 1e-12
    assert np.array_equal(yd.cpu().numpy(), y1)
    bad = y1.copy()
    bad[:, 0] += 3000 * PSI
    chosen, cnv = g.guess_select(yd, g.state(y0), g.state(bad), dt)
    assert chosen == 0 and cnv[1] > cnv[0]
    assert np.array_equal(yd.cpu().numpy(), y0)


def _train_on_trajectory(opm, g, states, steps, lr=2e-3, seed=0):
    net = opm.GuessNet(seed=seed)
    ys = [g.state(s) for s in states]
    for it in range(steps):
        k = it % (len(ys) - 1)
        g.guess_train_step(net, ys[k], ys[max(k - 1, 0)], ys[k + 1], lr)
    torch.cuda.synchronize()
    return net


def _waterflood_case():
    return cases.box_case(16, 14, 4, seed=23, dx=150 * cases.FT, dy=150 * cases.FT,
                          median_md=100.0, sigma_ln=1.0,
                          wells=[Well("I", cases.WELL_RATE_INJ, [(2, 2, k) for k in range(4)],
                                      1000 * STB / DAY),
                                 Well("P", cases.WELL_BHP_PROD, [(13, 11, 0)], 3000 * PSI),
                                 Well("P2", cases.WELL_BHP_PROD, [(13, 2, 0)], 3000 * PSI)],
                          report_dt=[10 * DAY] * 6, name="guess_waterflood")


@pytest.mark.parametrize("kind", ["extrapolation", "trained"])
@pytest.mark.parametrize("which", ["gas", "waterflood"])
def test_advance_with_guess_matches_oracle(opm, which, kind):
    """Converged states started from the guess match the oracle simulator
    (which starts every step from the previous state) to the path's bar."""
    case = _guess_case() if which == "gas" else _waterflood_case()
    g = opm.GpuModel(case)
    m = oracle.Model(case)
    states, _ = m.run()
    if kind == "trained":
        traj = [case.initial_state()] + [s for s in states]
        net = _train_on_trajectory(opm, g, traj, 300)
    else:   # zero correction: the guess is the linear extrapolation
        net = opm.GuessNet(np.zeros(opm.GUESS_PARAMS, np.float32))
    y = g.initial_state()
    y_nm1 = g.initial_state()
    used = []
    for k, dt in enumerate(case.report_dt):
        prev = y.clone()
        st, rep, u = g.advance_guess(y, y_nm1, dt, net)
        assert st == 0, (k, rep.as_dict())
        used.append(u)
        y_nm1 = prev
        yk = y.cpu().numpy()
        ref = states[k]
        assert np.max(np.abs(yk[:, 0] - ref[:, 0]) / np.abs(ref[:, 0])) <= 1e-6, k
        assert np.max(np.abs(yk[:, 1:] - ref[:, 1:])) <= 1e-6, k
        assert max(rep.cnv) <= case.tol_cnv and max(rep.mb) <= case.tol_mb
    print(which, kind, "guess taken", used)
    assert all(u in (0, 1, 2) for u in used)
    if which == "waterflood" and kind == "extrapolation":
        # the start really came from the guess at least once (1 and 2 are the
        # same state for a zero correction; the learned slot wins the tie)
        assert sum(1 for u in used if u) >= 1


def test_advance_guess_without_net_is_advance(opm):
    case = _guess_case()
    g = opm.GpuModel(case)
    y1 = g.initial_state()
    y2 = g.initial_state()
    for dt in case.report_dt[:2]:
        st1, r1 = g.advance(y1, dt)
        st2, r2, used = g.advance_guess(y2, None, dt, None)
        assert st1 == st2 == 0 and used == 0
        assert r1.newton_its == r2.newton_its and r1.lin_its == r2.lin_its
        assert torch.equal(y1, y2)


def test_guess_invalid_arguments(opm):
    L = opm._guess_lib()
    assert L.opm_guess_conv(0, 1, 1, None, None, None, 1, None, None, None) == opm.EINVAL
    assert L.opm_guess_conv_backward_bytes(0, 2, 2) == 0
    x = torch.zeros((16, 16), dtype=torch.int16, device="cuda")
    grad = torch.zeros(opm.GUESS_LAYER, dtype=torch.float32, device="cuda")
    work = torch.zeros(64, dtype=torch.uint8, device="cuda")
    need = L.opm_guess_conv_backward_bytes(2, 2, 2)
    assert need > 64
    rc = L.opm_guess_conv_backward(2, 2, 2, x.data_ptr(), x.data_ptr(), None, None, None,
                                   grad.data_ptr(), work.data_ptr(), 64, None)
    assert rc == opm.EINVAL
    case = _guess_case()
    g = opm.GpuModel(case)
    net = opm.GuessNet()
    s = net.struct(g)
    s.nx = 3            # box smaller than the active cell count
    import ctypes
    assert L.opm_guess_work_bytes(g._pbp(), ctypes.byref(s)) == 0
    with pytest.raises(opm.OpmError):
        g.guess_train_step(net, g.initial_state(), g.initial_state(), g.initial_state(), -1.0)


def test_full_size_forward_parity(opm):
    """Layer-by-layer parity on the 100x100x50 box (every cell), the size of
    the learned-guess workload."""
    shape = (50, 100, 100)
    x = cases.guess_random_feats(shape, seed=31, channels=11)
    p = cases.guess_init_params(7)
    net = opm.GuessNet(p)
    h_dev = _bits_to_dev(x)
    h = x.astype(np.float64)
    for l in range(3):
        W, b = cn.split(p)[l]
        relu = l < 2
        out = opm.guess_conv(shape, h_dev, net.w_fwd(l), net.bias(l), relu)
        got = _dev_to_box(out, shape, bf16=relu)
        Wr = cn.bf16(W)
        z = cn.conv(h, Wr, b)
        S = cn.conv_abs(h, Wr, b)
        ref = np.maximum(z, 0.0) if relu else z
        tol = 1e-4 * S + (2.0 ** -8 * np.abs(ref) if relu else 0.0)
        assert np.all(np.abs(got - ref) <= tol), l
        h, h_dev = got, out
