"""Plain FP64 oracle of the convolutional flood surrogate (numpy).

TEST INFRASTRUCTURE ONLY: used by the tests (and the benchmark's checks),
never by the product path; it shares no code with the GPU kernels.

The surrogate is not part of the paper: it is a learned shortcut that advances
the flood state k finite-volume steps at once.  Network (channels-last, 3x3
kernels, zero padding, stride 1): input planes (h, hu, hv, z, occupancy)
and the depth the inflow adds over the block on the inflow cells, scaled by
fixed constants and padded with zeros to 16 channels -> 64 -> 64 ->
64 -> 64 -> 3, ReLU after the first four layers; the three outputs are the
scaled change of (h, hu, hv) over the k steps.  Loss: mean squared error over
all outputs.  Optimiser: Adam (Kingma & Ba 2015) on FP32 master weights.

Precision: the network keeps its weights, activations and the gradients
that flow between layers in BF16 and accumulates in FP32.  With bf16=True
the oracle rounds at exactly those points (weights are passed in already
rounded; each hidden activation after its ReLU, the loss gradient and each
input gradient of a layer are rounded to BF16, round-to-nearest-even through
FP32) and computes everything else in FP64; with bf16=False it is the plain
FP64 network.

Everything here is the definition written out with plain loops over the nine
kernel taps and one matrix product per tap (a library primitive as a step).
"""
from __future__ import annotations

import numpy as np

CIN0 = 16                      # first layer input channels (5 used + 11 zero)
WIDTH = 64
LAYERS = [(CIN0, WIDTH), (WIDTH, WIDTH), (WIDTH, WIDTH), (WIDTH, WIDTH), (WIDTH, 3)]
# fixed input / output scales: h, hu, hv, z, occupancy  ->  O(1) values
IN_SCALE = np.array([1.0, 1.0, 1.0, 1.0 / 3.0, 0.25, 1.0] + [0.0] * 10)
N_IN = 6                       # used input channels: h, hu, hv, z, occupancy, inflow depth
OUT_SCALE = np.array([0.05, 0.05, 0.05])     # scaled change of (h, hu, hv) over k steps


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), through FP32: keep the
    upper 16 bits of the FP32 pattern after adding half of the dropped part's
    unit, plus one when the kept part is odd."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(f.shape)


def init_params(seed: int = 0):
    """He-normal weights [cout][3][3][cin] and zero biases, FP64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for cin, cout in LAYERS:
        std = np.sqrt(2.0 / (9 * cin))
        w = rng.normal(0.0, std, size=(cout, 3, 3, cin))
        if cin == CIN0:
            w[..., N_IN:] = 0.0
        params.append((w, np.zeros(cout)))
    return params


def conv3x3(x, w, b):
    """y[n, i, j, o] = b[o] + sum_{dy, dx, c} w[o, dy, dx, c] x[n, i+dy-1, j+dx-1, c],
    zero outside the image.  x: [N, H, W, Cin], w: [Cout, 3, 3, Cin]."""
    N, H, W, Ci = x.shape
    xp = np.zeros((N, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1, :] = x
    y = np.zeros((N, H, W, w.shape[0])) + b
    for dy in range(3):
        for dx in range(3):
            y += xp[:, dy:dy + H, dx:dx + W, :] @ w[:, dy, dx, :].T
    return y


def conv3x3_backward(x, w, dy):
    """Gradients of conv3x3 with respect to x, w and b for upstream dy."""
    N, H, W, Ci = x.shape
    xp = np.zeros((N, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1, :] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + H, kx:kx + W, :]
            dw[:, ky, kx, :] = np.einsum("nhwo,nhwc->oc", dy, patch)
            dxp[:, ky:ky + H, kx:kx + W, :] += dy @ w[:, ky, kx, :]
    db = dy.sum(axis=(0, 1, 2))
    return dxp[:, 1:-1, 1:-1, :], dw, db


def _round(a, bf16):
    return bf16_round(a) if bf16 else a


def forward(params, x, bf16=False):
    """Returns the output and the per-layer inputs / pre-activations."""
    acts, pres = [], []
    a = x
    for li, (w, b) in enumerate(params):
        acts.append(a)
        z = conv3x3(a, w, b)
        pres.append(z)
        a = _round(np.maximum(z, 0.0), bf16) if li < len(params) - 1 else z
    return a, acts, pres


def loss_and_grads(params, x, target, bf16=False):
    """MSE loss over all outputs and its gradients (list of (dw, db))."""
    y, acts, pres = forward(params, x, bf16)
    diff = y - target
    loss = float(np.mean(diff * diff))
    g = _round(2.0 * diff / diff.size, bf16)
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        w, _ = params[li]
        if li < len(params) - 1:
            g = g * (pres[li] > 0.0)
        dxl, dw, db = conv3x3_backward(acts[li], w, g)
        grads[li] = (dw, db)
        g = _round(dxl, bf16)
    return loss, grads


def adam_update(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), returns (param, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v


def pack_input(h, hu, hv, z, occ, inflow=None):
    """Scaled channels-last input [H, W, 16] from the state planes.  inflow:
    (side, c0, c1, depth) puts the block's inflow depth on the boundary cells
    of the inflow segment (sides W, E, S, N = 0, 1, 2, 3)."""
    x = np.zeros(h.shape + (CIN0,))
    for c, plane in enumerate((h, hu, hv, z, occ)):
        x[..., c] = plane * IN_SCALE[c]
    if inflow is not None and inflow[0] >= 0:
        side, c0, c1, depth = inflow
        ny, nx = h.shape
        if side == 2:
            x[0, c0:c1, 5] = depth * IN_SCALE[5]
        elif side == 3:
            x[ny - 1, c0:c1, 5] = depth * IN_SCALE[5]
        elif side == 0:
            x[c0:c1, 0, 5] = depth * IN_SCALE[5]
        else:
            x[c0:c1, nx - 1, 5] = depth * IN_SCALE[5]
    return x


def make_target(h0, hu0, hv0, h1, hu1, hv1):
    """Training target [H, W, 3]: the change of (h, hu, hv) over the k steps
    divided by OUT_SCALE."""
    return np.stack([(h1 - h0) / OUT_SCALE[0], (hu1 - hu0) / OUT_SCALE[1],
                     (hv1 - hv0) / OUT_SCALE[2]], axis=-1)


def apply_output(h, hu, hv, y, h_dry=1e-5, h_snap=1e-3):
    """State after the surrogate call: U + OUT_SCALE * y, depth kept >= 0; a
    cell that was dry stays dry unless the update puts at least h_snap on it;
    no discharge in cells left dry (h <= h_dry), as in the flood update."""
    hn = np.maximum(h + OUT_SCALE[0] * y[..., 0], 0.0)
    hn = np.where((h <= h_dry) & (hn < h_snap), 0.0, hn)
    wet = hn > h_dry
    qx = np.where(wet, hu + OUT_SCALE[1] * y[..., 1], 0.0)
    qy = np.where(wet, hv + OUT_SCALE[2] * y[..., 2], 0.0)
    return hn, qx, qy


def hazard_class32(h, qx, qy, h_dry, thr):
    """Hazard class of Table 1 (0 dry, 1 low .. 4 highest) from float32 states,
    decided in float32: HR = (max(|u|, |v|) + 0.5) h against the thresholds."""
    h = np.asarray(h, np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = np.asarray(qx, np.float32) / h
        v = np.asarray(qy, np.float32) / h
        hr = (np.maximum(np.abs(u), np.abs(v)) + np.float32(0.5)) * h
    t = [np.float32(x) for x in thr]
    cls = np.where(hr < t[0], 1, np.where(hr < t[1], 2, np.where(hr < t[2], 3, 4)))
    return np.where(h > np.float32(h_dry), cls, 0)


def judge(x, y, state, nx, ny, dx, dy, a, b, tol, h_dry, thr, exited=1, stride=1, select=None, hr_margin=0.0,
          h_margin=0.0):
    """Judge of a surrogate flood state a = (h, qx, qy) against a
    finite-volume state b at the cells of the judged agents still in the
    domain: every stride-th agent, and with a selection state select = (h, qx,
    qy) also every agent whose cell there has a depth within h_margin of the
    dry threshold or a hazard rate within hr_margin of a threshold of thr
    (decided in float32, as the GPU decides it).  Returns (judged agents whose
    depth differs by more than tol or whose hazard class differs, largest
    depth difference, judged agents).  Cells: floor(x / dx) in float32,
    clamped to the grid."""
    x = np.asarray(x, np.float32)
    y = np.asarray(y, np.float32)
    idx = np.arange(len(x))
    i = np.clip(np.floor(x / np.float32(dx)), 0, nx - 1).astype(np.int64)
    j = np.clip(np.floor(y / np.float32(dy)), 0, ny - 1).astype(np.int64)
    pick = idx % stride == 0
    if select is not None:
        hs, qxs, qys = (np.asarray(f, np.float32)[j, i] for f in select)
        with np.errstate(divide="ignore", invalid="ignore"):
            v = np.maximum(np.abs(qxs / hs), np.abs(qys / hs)).astype(np.float32)
            hr = ((v + np.float32(0.5)) * hs).astype(np.float32)
        near_dry = ~(hs > np.float32(h_dry) + np.float32(h_margin))
        near_thr = np.zeros(len(x), bool)
        for t in thr:
            near_thr |= np.abs(hr - np.float32(t)) < np.float32(hr_margin)
        pick |= near_dry | near_thr
    keep = (np.asarray(state) != exited) & pick
    i, j = i[keep], j[keep]
    if i.size == 0:
        return 0, 0.0, 0
    ha, qxa, qya = (np.asarray(f, np.float32)[j, i] for f in a)
    hb, qxb, qyb = (np.asarray(f, np.float32)[j, i] for f in b)
    d = np.abs(ha - hb)
    bad = (d > np.float32(tol)) | (hazard_class32(ha, qxa, qya, h_dry, thr)
                                    != hazard_class32(hb, qxb, qyb, h_dry, thr))
    return int(bad.sum()), float(d.max()), int(i.size)
