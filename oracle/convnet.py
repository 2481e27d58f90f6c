"""Plain numpy oracle of the learned Newton initial guess.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (and nothing in the GPU
library).  Everything is FP64 except where the network's stated storage
precision applies: weights and stored activations are BF16 (round to nearest
even, through FP32 as the kernels do), sums are exact-order-free FP64 here.

The network (not part of the paper; the paper's Newton method, sec. 2.3,
starts every step from the previous state): three 3-D convolution layers
with 3x3x3 kernels and 16 channels, zero padding at the faces of the
nx*ny*nz box, ReLU after layers 1 and 2.  Arrays are channels-last
[nz, ny, nx, 16]; weights W[t][out][in] with tap t = 9 (dz+1) + 3 (dy+1) +
(dx+1) reading the box cell (x+dx, y+dy, z+dz); the parameter vector holds
W_0, b_0, W_1, b_1, W_2, b_2.  The predicted step is the last step
y_n - y_{n-1} (a skip connection: linear extrapolation) plus the network's
correction of the two saturations (output channels 1 and 2; the pressure
keeps the extrapolation and output channel 0 is unused); training minimises
the mean squared error of the two saturation outputs against the scaled
correction with Adam (Kingma and Ba, 2015).
"""
from __future__ import annotations

import numpy as np

CH = 16
TAPS = 27
LAYER_W = TAPS * CH * CH
LAYER = LAYER_W + CH
PARAMS = 3 * LAYER

PSI = 6894.757293168
P0 = 4800.0 * PSI
PS = 1000.0 * PSI
QS = 86400.0 / 10.0
MU_REF = 1e-3
DPS = 100.0 * PSI
DSS = 0.1
MILLIDARCY = 9.869233e-16


# ----------------------------------------------------------------- BF16
def to_bf16_bits(x) -> np.ndarray:
    """FP64/FP32 -> FP32 (nearest even) -> BF16 bits (nearest even)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    r = np.where(nan, ((u >> 16) | 0x40) & 0xFFFF, r)
    return r.astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(
        np.float64)


def bf16(x) -> np.ndarray:
    """Value of x after storage in BF16."""
    return from_bf16_bits(to_bf16_bits(x))


# ---------------------------------------------------------- convolution
def tap_offset(t: int):
    """(dx, dy, dz) of tap t."""
    return t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1


def _shifted(x: np.ndarray, dx: int, dy: int, dz: int) -> np.ndarray:
    """s[z, y, x] = x[z+dz, y+dy, x+dx], zero outside the box."""
    nz, ny, nx = x.shape[:3]
    xp = np.zeros((nz + 2, ny + 2, nx + 2) + x.shape[3:], dtype=np.float64)
    xp[1:-1, 1:-1, 1:-1] = x
    return xp[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]


def conv(x: np.ndarray, W: np.ndarray, b=None) -> np.ndarray:
    """out[c][o] = b[o] + sum_t sum_i x[c + off_t][i] W[t][o][i]."""
    out = np.zeros(x.shape[:3] + (W.shape[1],))
    for t in range(TAPS):
        out += _shifted(x, *tap_offset(t)) @ W[t].T
    if b is not None:
        out += b
    return out


def conv_transpose(d: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Adjoint of conv in x: g[c][i] = sum_t sum_o d[c - off_t][o] W[t][o][i]."""
    out = np.zeros(d.shape[:3] + (W.shape[2],))
    for t in range(TAPS):
        dx, dy, dz = tap_offset(t)
        out += _shifted(d, -dx, -dy, -dz) @ W[t]
    return out


def conv_weight_grad(x: np.ndarray, d: np.ndarray):
    """Adjoint of conv in (W, b): dW[t][o][i] = sum_c d[c][o] x[c + off_t][i],
    db[o] = sum_c d[c][o]."""
    dW = np.zeros((TAPS, d.shape[3], x.shape[3]))
    df = d.reshape(-1, d.shape[3])
    for t in range(TAPS):
        dW[t] = df.T @ _shifted(x, *tap_offset(t)).reshape(-1, x.shape[3])
    return dW, df.sum(axis=0)


def conv_abs(x: np.ndarray, W: np.ndarray, b=None) -> np.ndarray:
    """sum of |terms| of conv (scale for rounding tolerances)."""
    return conv(np.abs(x), np.abs(W), None if b is None else np.abs(b))


# -------------------------------------------------------------- network
def split(params: np.ndarray):
    """[(W_l [27][16][16], b_l [16])] for l = 0, 1, 2."""
    p = np.asarray(params, dtype=np.float64)
    out = []
    for l in range(3):
        base = l * LAYER
        out.append((p[base:base + LAYER_W].reshape(TAPS, CH, CH), p[base + LAYER_W:base + LAYER]))
    return out


def forward(feats: np.ndarray, params: np.ndarray, rounded: bool = True):
    """Activations (a0, a1, a2) and the output of the network.  rounded: BF16
    weights and stored activations as in the kernels; False gives the exact
    FP64 network (for derivative checks)."""
    r = bf16 if rounded else (lambda v: np.asarray(v, dtype=np.float64))
    layers = split(params)
    a0 = r(feats)
    acts = [a0]
    h = a0
    for l, (W, b) in enumerate(layers):
        z = conv(h, r(W), b)
        if l < 2:
            h = r(np.maximum(z, 0.0))
            acts.append(h)
        else:
            out = z
    return acts, out


def targets(y_n: np.ndarray, y_nm1: np.ndarray, y_next: np.ndarray) -> np.ndarray:
    """Scaled correction of the step to the linearly extrapolated one per
    active cell, (y_next - y_n) - (y_n - y_{n-1}), as (dp / 100 psi,
    ds_w / 0.1, ds_g / 0.1)."""
    y_n = np.asarray(y_n, dtype=np.float64)
    d = (np.asarray(y_next, dtype=np.float64) - y_n) - (y_n - np.asarray(y_nm1, dtype=np.float64))
    return np.stack([d[:, 0] / DPS, d[:, 1] / DSS, d[:, 2] / DSS], axis=1)


def to_box(v: np.ndarray, cell_box: np.ndarray, shape, ch: int = CH) -> np.ndarray:
    """Scatter per-cell rows into a zero [nz, ny, nx, ch] box."""
    nz, ny, nx = shape
    box = np.zeros((nz * ny * nx, ch))
    box[np.asarray(cell_box), :v.shape[1]] = v
    return box.reshape(nz, ny, nx, ch)


def away_from_wells(feats_box: np.ndarray, cell_box: np.ndarray) -> np.ndarray:
    """Active cells where corrections apply: neither the cell nor any of its
    26 box neighbours has a non-zero well channel (7-10) in the feature box."""
    w = np.any(feats_box[..., 7:11] != 0.0, axis=3)
    near = np.zeros_like(w)
    for t in range(TAPS):
        near |= _shifted(w.astype(np.float64), *tap_offset(t)) != 0.0
    return ~near.ravel()[np.asarray(cell_box)]


def loss_and_dout(out: np.ndarray, tgt: np.ndarray, cell_box: np.ndarray, rounded: bool = True,
                  free=None):
    """Squared error of the two saturation outputs (channels 1 and 2; the
    pressure output, channel 0, is neither trained nor used) summed over the
    active cells in `free` (all if None) and divided by 2 n_cells, and dL/d out
    as a box (BF16 when rounded)."""
    n = tgt.shape[0]
    o = out.reshape(-1, out.shape[3])[np.asarray(cell_box), :3]
    e = o - tgt
    e[:, 0] = 0.0
    if free is not None:
        e = np.where(np.asarray(free)[:, None], e, 0.0)
    loss = float(np.sum(e * e) / (2.0 * n))
    g = 2.0 * e / (2.0 * n)
    if rounded:
        g = bf16(g)
    return loss, to_box(g, cell_box, out.shape[:3])


def backward(acts, dout: np.ndarray, params: np.ndarray, rounded: bool = True) -> np.ndarray:
    """Gradient of the loss w.r.t. the parameter vector, given the stored
    activations and dL/d(output of layer 3)."""
    r = bf16 if rounded else (lambda v: np.asarray(v, dtype=np.float64))
    layers = split(params)
    grad = np.zeros(PARAMS)
    d = dout
    for l in (2, 1, 0):
        dW, db = conv_weight_grad(acts[l], d)
        grad[l * LAYER:l * LAYER + LAYER_W] = dW.ravel()
        grad[l * LAYER + LAYER_W:(l + 1) * LAYER] = db
        if l > 0:
            W = r(layers[l][0])
            d = r(np.where(acts[l] > 0.0, conv_transpose(d, W), 0.0))
    return grad


def adam(w, g, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step is 1-based); returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# -------------------------------------------------- features and guess
def features(case, y_n, y_nm1, cell_box, conn_cell, conn_wi, conn_well, rounded: bool = True):
    """Layer-0 input box: (p_n - 4800 psi)/1000 psi, s_w, s_g of y_n, the
    last change (p_n - p_{n-1})/100 psi, (s_n - s_{n-1})/0.1 of both
    saturations, log10(k_h / 1 mD) - 2, injection rates of water, oil and gas per
    10 m^3/day (a rate injector's target split over its connections in
    proportion to WI), ln(1 + sum WI (p_n - p_bhp)^+ / 1 cP per 10 m^3/day)
    of producers; other channels zero."""
    y_n = np.asarray(y_n, dtype=np.float64)
    y_nm1 = np.asarray(y_nm1, dtype=np.float64)
    n = y_n.shape[0]
    f = np.zeros((n, CH))
    f[:, 0] = (y_n[:, 0] - P0) / PS
    f[:, 1:3] = y_n[:, 1:3]
    f[:, 3] = (y_n[:, 0] - y_nm1[:, 0]) / DPS
    f[:, 4:6] = (y_n[:, 1:3] - y_nm1[:, 1:3]) / DSS
    perm = np.asarray(case.perm_h, dtype=np.float64).ravel()[np.asarray(cell_box)]
    f[:, 6] = np.log10(perm / MILLIDARCY) - 2.0
    inj = np.zeros((n, 3))
    prod = np.zeros(n)
    wi_sum = np.zeros(len(case.wells))
    for k in range(len(conn_cell)):
        wi_sum[conn_well[k]] += conn_wi[k]
    for k in range(len(conn_cell)):
        w = case.wells[conn_well[k]]
        c = conn_cell[k]
        if w.kind == 0:      # rate injector
            inj[c, w.phase] += w.target * conn_wi[k] / wi_sum[conn_well[k]]
        else:
            dd = y_n[c, 0] - w.target
            if dd > 0.0:
                prod[c] += conn_wi[k] * dd
    f[:, 7:10] = inj * QS
    f[:, 10] = np.log1p(prod / MU_REF * QS)
    box = to_box(f, cell_box, (case.nz, case.ny, case.nx))
    return bf16(box) if rounded else box


def apply_guess(y_n: np.ndarray, y_nm1: np.ndarray, out: np.ndarray,
                cell_box: np.ndarray, free=None) -> np.ndarray:
    """y_n + (y_n - y_{n-1}), plus the network's correction of the two
    saturations (in units of 0.1; the pressure keeps the extrapolation), the
    correction only in cells of `free` (all if None) and only where all three
    outputs are finite; saturations clamped to [0, 1], s_g lowered so that
    s_w + s_g <= 1."""
    y_n = np.asarray(y_n, dtype=np.float64)
    e = y_n + (y_n - np.asarray(y_nm1, dtype=np.float64))
    o = out.reshape(-1, out.shape[3])[np.asarray(cell_box), :3]
    ok = np.all(np.isfinite(o), axis=1)
    if free is not None:
        ok &= np.asarray(free)
    o = np.where(ok[:, None], o, 0.0)
    p = e[:, 0]
    sw = np.clip(e[:, 1] + DSS * o[:, 1], 0.0, 1.0)
    sg = np.clip(e[:, 2] + DSS * o[:, 2], 0.0, 1.0)
    sg = np.where(sw + sg > 1.0, 1.0 - sw, sg)
    return np.stack([p, sw, sg], axis=1)
