"""GPU parity of the BF16 MFMA surrogate kernels against the FP64 oracle.

The GPU keeps weights, activations and inter-layer gradients in BF16 and
accumulates in FP32.  The oracle rounds at the same points (bf16=True) and
computes the rest in FP64; against it the bars are forward relative L2
<= 5e-3 and per-tensor gradients cosine >= 0.9999 and relative L2 <= 1e-2
(what remains is FP32 against FP64 accumulation, which can move a BF16
rounding by one unit).  Against the plain FP64 network (bf16=False) the bars
are those of BF16 rounding compounded over four layers of backward pass:
forward relative L2 <= 2e-2, gradients cosine >= 0.995 and relative L2
<= 0.1 (the first layer's weight gradient is a sum with strong cancellation;
a CPU run with BF16 rounding alone gives 3-6e-2 there)."""
import numpy as np
import pytest
import torch

from oracle import surrogate_oracle as S
from paper_1908_05232_amd import fps
from tests.gpu_util import say

pytestmark = pytest.mark.gpu
COUT_GPU = [64, 64, 64, 64, 16]
# element-wise bar of a gradient against the oracle with the same BF16
# rounding points, relative to the largest element of its tensor: the FP32
# sums may move an inter-layer BF16 rounding by one unit (2^-8 relative) at
# a few pixels, whose share of a weight-gradient sum over the image is far
# below that unit; measured up to 5e-4 (first layer) on the multi-tile case
ELEM_TOL = 5e-3


bf16_round = S.bf16_round


def pack(params):
    """Oracle parameters -> packed FP32 vector with the GPU's channel padding."""
    out = []
    for li, (w, b) in enumerate(params):
        co = COUT_GPU[li]
        wp = np.zeros((co,) + w.shape[1:])
        wp[: w.shape[0]] = w
        bp = np.zeros(co)
        bp[: b.shape[0]] = b
        out += [wp.reshape(-1), bp]
    return np.concatenate(out)


def unpack(vec, params):
    res, o = [], 0
    for li, (w, b) in enumerate(params):
        co = COUT_GPU[li]
        nw = co * 9 * w.shape[3]
        wp = vec[o:o + nw].reshape((co,) + w.shape[1:])
        o += nw
        bp = vec[o:o + co]
        o += co
        res.append((wp[: w.shape[0]], bp[: b.shape[0]]))
    return res


def make_case(seed, n, H, W):
    rng = np.random.default_rng(seed)
    params = [(bf16_round(w), bf16_round(rng.normal(0, 0.05, b.shape))) for w, b in S.init_params(seed)]
    x = np.zeros((n, H, W, S.CIN0))
    x[..., :5] = rng.uniform(-1, 1, (n, H, W, 5))
    x = bf16_round(x)
    target = rng.normal(0, 0.5, (n, H, W, 3))
    return params, x, target


def to_dev(params, x, target):
    xt = torch.tensor(x, dtype=torch.float32).bfloat16().cuda().contiguous()
    tt = torch.zeros(target.shape[:3] + (4,), dtype=torch.float32)
    tt[..., :3] = torch.tensor(target)
    return torch.tensor(pack(params), dtype=torch.float32).cuda(), xt, tt.cuda().contiguous()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def cosine(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


def test_forward_matches_oracle():
    params, x, target = make_case(1, 2, 16, 64)
    sur = fps.Surrogate(2, 16, 64)
    p, xt, _ = to_dev(params, x, target)
    sur.set_params(p)
    y = sur.forward(xt).cpu().numpy()
    yb, _, _ = S.forward(params, x, bf16=True)
    yo, _, _ = S.forward(params, x)
    eb, eo = rel_l2(y[..., :3], yb), rel_l2(y[..., :3], yo)
    say(f"surrogate forward rel L2 {eb:.2e} (bf16 points), {eo:.2e} (fp64)")
    assert eb <= 5e-3 and eo <= 2e-2
    assert np.all(y[..., 3] == 0.0)


@pytest.mark.parametrize("seed", [2, 5])
def test_gradients_match_oracle(seed):
    params, x, target = make_case(seed, 2, 16, 64)
    sur = fps.Surrogate(2, 16, 64)
    p, xt, tt = to_dev(params, x, target)
    sur.set_params(p)
    loss, g = sur.gradients(xt, tt)
    lb, gb = S.loss_and_grads(params, x, target, bf16=True)
    lo, go = S.loss_and_grads(params, x, target)
    assert float(loss.item()) == pytest.approx(lb, rel=5e-3)
    gg = unpack(g.cpu().numpy().astype(np.float64), params)
    for li in range(len(gg)):
        for ref, cos_min, rel_max, tag in ((gb, 0.9999, 1e-2, "bf16"), (go, 0.995, 0.1, "fp64")):
            (dw, db), (dwo, dbo) = gg[li], ref[li]
            if li == 0:
                dw, dwo = dw[..., :5], dwo[..., :5]       # zero input channels carry no gradient
            c, e = cosine(dw, dwo), rel_l2(dw, dwo)
            cb, eb = cosine(db, dbo), rel_l2(db, dbo)
            say(f"layer {li + 1} vs {tag}: dW cos {c:.6f} rel {e:.2e}; db cos {cb:.6f} rel {eb:.2e}")
            assert c >= cos_min and e <= rel_max and cb >= cos_min and eb <= rel_max


def test_multi_tile_gradients_match_oracle():
    """Every block walks several tiles: the kernels' grid-stride paths (next
    tile prefetched during the matrix work, LDS re-deposit, partial weight
    gradients accumulated over tiles) against the oracle, element by element.
    3 images of 48 x 96 make 27 convolution tiles (16 x 32 pixels) and 144
    weight-gradient tiles (4 x 8 positions of the 8-image group, 5 of the 8
    images past the batch); caps of 5 and 7 blocks give each block 5-6 and
    20-21 of them, the last block fewer (ragged).  The forward pass must not change at all under
    the caps, the gradients only by the grouping of their FP32 partial sums."""
    params, x, target = make_case(9, 3, 48, 96)
    sur = fps.Surrogate(3, 48, 96)
    p, xt, tt = to_dev(params, x, target)
    sur.set_params(p)
    y_one = sur.forward(xt).clone()
    _, g_one = sur.gradients(xt, tt)
    g_one = g_one.clone()
    sur.set_blocks(5, 7)
    y = sur.forward(xt)
    loss, g = sur.gradients(xt, tt)
    assert torch.equal(y, y_one)
    gn, g1 = g.cpu().numpy().astype(np.float64), g_one.cpu().numpy().astype(np.float64)
    regroup = float(np.abs(gn - g1).max() / np.abs(g1).max())
    say(f"capped vs one tile per block: max|dg| / max|g| = {regroup:.2e}")
    assert regroup <= 1e-5
    lb, gb = S.loss_and_grads(params, x, target, bf16=True)
    assert float(loss.item()) == pytest.approx(lb, rel=5e-3)
    yb, _, _ = S.forward(params, x, bf16=True)
    yerr = float(np.abs(y.cpu().numpy()[..., :3] - yb).max() / np.abs(yb).max())
    say(f"forward: max|dy| / max|y| = {yerr:.2e}")
    assert yerr <= 5e-3
    gg = unpack(gn, params)
    for li in range(len(gg)):
        (dw, db), (dwb, dbb) = gg[li], gb[li]
        if li == 0:
            dw, dwb = dw[..., :5], dwb[..., :5]       # zero input channels carry no gradient
        ew = float(np.abs(dw - dwb).max() / np.abs(dwb).max())
        eb = float(np.abs(db - dbb).max() / np.abs(dbb).max())
        c, e = cosine(dw, dwb), rel_l2(dw, dwb)
        say(f"layer {li + 1}: dW max|d| / max|ref| {ew:.2e} (cos {c:.6f}, rel L2 {e:.2e}); "
            f"db max|d| / max|ref| {eb:.2e}")
        assert ew <= ELEM_TOL and eb <= ELEM_TOL
        assert c >= 0.9999 and e <= 1e-2


def test_gradients_over_two_image_groups_match_oracle():
    """The weight gradient takes the batch eight images at a time (the k
    index of its matrix products runs over the images of one position): 9
    images make one full group and one with a single image and seven empty
    slots.  Element by element against the oracle with the same BF16
    rounding points, as the multi-tile test."""
    params, x, target = make_case(13, 9, 16, 64)
    sur = fps.Surrogate(9, 16, 64)
    p, xt, tt = to_dev(params, x, target)
    sur.set_params(p)
    loss, g = sur.gradients(xt, tt)
    lb, gb = S.loss_and_grads(params, x, target, bf16=True)
    assert float(loss.item()) == pytest.approx(lb, rel=5e-3)
    gg = unpack(g.cpu().numpy().astype(np.float64), params)
    for li in range(len(gg)):
        (dw, db), (dwb, dbb) = gg[li], gb[li]
        if li == 0:
            dw, dwb = dw[..., :5], dwb[..., :5]       # zero input channels carry no gradient
        ew = float(np.abs(dw - dwb).max() / np.abs(dwb).max())
        eb = float(np.abs(db - dbb).max() / np.abs(dbb).max())
        say(f"9 images, layer {li + 1}: dW max|d| / max|ref| {ew:.2e}, db {eb:.2e}")
        assert ew <= ELEM_TOL and eb <= ELEM_TOL
        assert cosine(dw, dwb) >= 0.9999 and rel_l2(dw, dwb) <= 1e-2


def test_training_reduces_loss_and_matches_adam():
    params, x, target = make_case(3, 2, 16, 64)
    sur = fps.Surrogate(2, 16, 64)
    p, xt, tt = to_dev(params, x, target)
    sur.set_params(p)
    losses = []
    for _ in range(60):
        losses.append(float(sur.train_step(xt, tt, 2e-3).item()))
    say(f"loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.5 * losses[0]
    # one Adam step from fresh moments moves every weight with a gradient by about lr
    sur.set_params(p)
    _, g = sur.gradients(xt, tt)
    sur.train_step(xt, tt, 1e-3)
    delta = (sur.get_params() - p).cpu().numpy()
    gn = g.cpu().numpy()
    big = np.abs(gn) > 1e-6
    assert np.allclose(np.abs(delta[big]), 1e-3, rtol=0.05)
    assert np.all(delta[gn == 0.0] == 0.0)


def _planes(rng, H, W):
    h = rng.uniform(0, 1.5, (H, W)).astype(np.float32)
    h[rng.uniform(size=(H, W)) < 0.3] = 0.0
    hu = rng.normal(0, 0.5, (H, W)).astype(np.float32)
    hv = rng.normal(0, 0.5, (H, W)).astype(np.float32)
    return h, hu, hv


def test_pack_target_apply_match_oracle():
    rng = np.random.default_rng(11)
    H, W = 24, 37
    h, hu, hv = _planes(rng, H, W)
    z = rng.uniform(-1, 3, (H, W)).astype(np.float32)
    occ = rng.integers(0, 6, (H, W)).astype(np.int32)
    dev = [torch.tensor(a).cuda() for a in (h, hu, hv, z, occ)]
    inflow = (2, 5, 20, 0.37)
    x = fps.sur_pack(*dev, inflow=inflow).float().cpu().numpy()
    xo = S.pack_input(*(a.astype(np.float64) for a in (h, hu, hv, z, occ)), inflow=inflow)
    assert np.count_nonzero(xo[..., 5]) == 15
    xr = bf16_round(xo)
    keep = [0, 1, 2, 4] + list(range(5, 16))
    assert np.array_equal(x[..., keep], xr[..., keep])
    assert np.allclose(x[..., 3], xr[..., 3], rtol=2.0 ** -7, atol=0)   # z / 3: one bf16 ulp
    x0 = fps.sur_pack(*dev[:4]).float().cpu().numpy()       # no occupancy, no inflow
    assert np.all(x0[..., 4:] == 0) and np.array_equal(x0[..., :4], x[..., :4])
    for side, c0, c1 in ((0, 3, 9), (1, 0, 24), (3, 30, 37)):
        xs = fps.sur_pack(*dev, inflow=(side, c0, c1, 0.2)).float().cpu().numpy()
        xso = S.pack_input(*(a.astype(np.float64) for a in (h, hu, hv, z, occ)), inflow=(side, c0, c1, 0.2))
        assert np.array_equal(xs[..., 5], bf16_round(xso[..., 5]))
    # target and apply: U1 reproduced from U0 and its target (within FP32 rounding)
    h1, hu1, hv1 = _planes(rng, H, W)
    s0 = [torch.tensor(a).cuda() for a in (h, hu, hv)]
    s1 = [torch.tensor(a).cuda() for a in (h1, hu1, hv1)]
    t = fps.sur_make_target(s0, s1).cpu().numpy()
    to = S.make_target(*(a.astype(np.float64) for a in (h, hu, hv, h1, hu1, hv1)))
    assert np.allclose(t[..., :3], to, rtol=1e-6, atol=1e-6) and np.all(t[..., 3] == 0)
    y = torch.tensor(t).cuda()
    fps.sur_apply(y, *s0)
    got = [a.cpu().numpy() for a in s0]
    want = S.apply_output(h.astype(np.float64), hu.astype(np.float64), hv.astype(np.float64),
                          t[..., :3].astype(np.float64))
    for g, w in zip(got, want):
        assert np.allclose(g, w, rtol=0, atol=2e-6)
    assert np.all(got[1][got[0] <= 1e-5] == 0) and np.all(got[0] >= 0)


def test_judge_matches_oracle():
    rng = np.random.default_rng(12)
    nx, ny, dx, dy = 53, 41, 0.5, 0.5
    b = _planes(rng, ny, nx)
    a = tuple(p + rng.normal(0, 0.01, p.shape).astype(np.float32) * (rng.uniform(size=p.shape) < 0.2)
              for p in b)
    a = (np.maximum(a[0], 0).astype(np.float32), a[1], a[2])
    na = 3001
    x = rng.uniform(-1, nx * dx + 1, na).astype(np.float32)
    y = rng.uniform(-1, ny * dy + 1, na).astype(np.float32)
    st = rng.integers(0, 3, na).astype(np.uint8)
    dv = lambda arr: torch.tensor(arr).cuda()
    for stride in (1, 3):
        want = S.judge(x, y, st, nx, ny, dx, dy, a, b, 0.01, 1e-5, (0.75, 1.5, 2.5), stride=stride)
        out = fps.sur_judge(dv(x), dv(y), dv(st), nx, ny, dx, dy, tuple(map(dv, a)), tuple(map(dv, b)),
                            stride=stride)
        got = fps.judge_result(out)
        say(f"judge stride {stride}: {got} oracle {want}")
        assert got == want and want[0] > 0
    # the sample plus the people near a class boundary of a selection state
    sel = _planes(np.random.default_rng(14), ny, nx)
    for stride, hrm, hm in ((50, 0.1, 0.01), (1000000, 0.05, 0.0), (7, 0.0, 0.02)):
        want = S.judge(x, y, st, nx, ny, dx, dy, a, b, 0.01, 1e-5, (0.75, 1.5, 2.5), stride=stride, select=sel,
                       hr_margin=hrm, h_margin=hm)
        out = fps.sur_judge(dv(x), dv(y), dv(st), nx, ny, dx, dy, tuple(map(dv, a)), tuple(map(dv, b)),
                            stride=stride, select=tuple(map(dv, sel)), hr_margin=hrm, h_margin=hm)
        got = fps.judge_result(out)
        plain = S.judge(x, y, st, nx, ny, dx, dy, a, b, 0.01, 1e-5, (0.75, 1.5, 2.5), stride=stride)
        say(f"judge stride {stride} + margins {hrm}, {hm}: {got} oracle {want} (sample alone: {plain[2]} judged)")
        assert got == want and want[2] > plain[2]
    # no agents -> (0, 0, 0); identical states -> nothing off
    out0 = fps.sur_judge(dv(x[:0]), dv(y[:0]), dv(st[:0]), nx, ny, dx, dy, tuple(map(dv, a)),
                         tuple(map(dv, b)))
    assert fps.judge_result(out0) == (0, 0.0, 0)
    same = fps.sur_judge(dv(x), dv(y), dv(st), nx, ny, dx, dy, tuple(map(dv, b)), tuple(map(dv, b)))
    assert fps.judge_result(same)[:2] == (0, 0.0)


def _cells(x, y, nx, ny, dx, dy):
    i = np.clip(np.floor(x / np.float32(dx)), 0, nx - 1).astype(np.int64)
    j = np.clip(np.floor(y / np.float32(dy)), 0, ny - 1).astype(np.int64)
    return i, j


def test_occupancy_and_judge_mask():
    rng = np.random.default_rng(13)
    nx, ny, dx, dy = 75, 50, 0.25, 0.25
    na = 4000
    x = rng.uniform(0, nx * dx, na).astype(np.float32)
    y = rng.uniform(0, ny * dy, na).astype(np.float32)
    role = (rng.uniform(size=na) < 0.1).astype(np.uint8)
    st = rng.integers(0, 3, na).astype(np.uint8)
    dv = lambda arr: torch.tensor(arr).cuda()
    occ = fps.sur_occupancy(dv(x), dv(y), dv(role), dv(st), nx, ny, dx, dy).cpu().numpy()
    i, j = _cells(x, y, nx, ny, dx, dy)
    keep = (role == 0) & (st == 0)
    want = np.zeros((ny, nx), np.int64)
    np.add.at(want, (j[keep], i[keep]), 1)
    assert np.array_equal(occ, want)
    halo, block, stride = 8, 16, 7
    m = fps.sur_judge_mask(dv(x), dv(y), dv(st), nx, ny, dx, dy, halo, block, stride=stride).cpu().numpy()
    wm = np.zeros(((ny + block - 1) // block, (nx + block - 1) // block), np.uint8)
    for a in range(0, na, stride):
        if st[a] == 1:
            continue
        wm[max(j[a] - halo, 0) // block:min(j[a] + halo, ny - 1) // block + 1,
           max(i[a] - halo, 0) // block:min(i[a] + halo, nx - 1) // block + 1] = 1
    assert np.array_equal(m, wm)
    # with a selection state: the region also covers the people near a class boundary
    # (a sparse sample, so that the extra people add blocks)
    stride = 1500
    m = fps.sur_judge_mask(dv(x), dv(y), dv(st), nx, ny, dx, dy, halo, block, stride=stride).cpu().numpy()
    sel = _planes(rng, ny, nx)
    m2 = fps.sur_judge_mask(dv(x), dv(y), dv(st), nx, ny, dx, dy, halo, block, stride=stride,
                            select=tuple(map(dv, sel)), hr_margin=0.1, h_margin=0.01).cpu().numpy()
    hs, qxs, qys = (p[j, i] for p in sel)
    with np.errstate(divide="ignore", invalid="ignore"):
        hr = ((np.maximum(np.abs(qxs / hs), np.abs(qys / hs)).astype(np.float32) + np.float32(0.5)) * hs)
    near = ~(hs > np.float32(1e-5) + np.float32(0.01))
    for t in (0.75, 1.5, 2.5):
        near |= np.abs(hr.astype(np.float32) - np.float32(t)) < np.float32(0.1)
    wm2 = np.zeros_like(wm)
    for a in range(na):
        if st[a] == 1 or not (a % stride == 0 or near[a]):
            continue
        wm2[max(j[a] - halo, 0) // block:min(j[a] + halo, ny - 1) // block + 1,
            max(i[a] - halo, 0) // block:min(i[a] + halo, nx - 1) // block + 1] = 1
    assert np.array_equal(m2, wm2) and m2.sum() > m.sum()


def test_judge_region_is_exact_inside():
    """k steps on a judge region equal k full steps (same fixed step) at cells
    at least k cells inside the region, bit for bit."""
    from paper_1908_05232_amd import inputs as I
    from tests.gpu_util import random_wet_dry
    sc = random_wet_dry(300, 170, 0.25, seed=21, bc=(0, 1, 0, 1), inflow=(2, 100, 140))
    sc.desc.dt_max = 0.001                     # below the CFL step of this state
    full, part = fps.Sim(sc), fps.Sim(sc)
    full.set_graph(0)
    part.set_graph(0)
    block, halo, k = 16, 8, 8
    rng = np.random.default_rng(3)
    na = 12
    x = rng.uniform(0, 300 * 0.25, na).astype(np.float32)
    y = rng.uniform(0, 170 * 0.25, na).astype(np.float32)
    st = np.zeros(na, np.uint8)
    dv = lambda arr: torch.tensor(arr).cuda()
    mask = fps.sur_judge_mask(dv(x), dv(y), dv(st), 300, 170, 0.25, 0.25, halo, block)
    part.set_judge_region(mask, block)
    for _ in range(2):                          # two blocks: stale values from the first stay outside
        full.step(k)
        part.step(k)
        assert full.diag()["dt_last"] == np.float32(0.001) and part.diag()["dt_last"] == np.float32(0.001)
        F, P = full.fields(), part.fields()
        i, j = _cells(x, y, 300, 170, 0.25, 0.25)
        for a, b in zip(F[:3], P[:3]):
            assert np.array_equal(a[j, i], b[j, i])
        # and every cell whose whole (2k+1)^2 neighbourhood lies in marked blocks
        mb = np.kron(mask.cpu().numpy(), np.ones((block, block), np.uint8))[:170, :300].astype(bool)
        from scipy.ndimage import binary_erosion
        inner = binary_erosion(mb, np.ones((2 * k + 1, 2 * k + 1), bool), border_value=1)
        for a, b in zip(F[:3], P[:3]):
            assert np.array_equal(a[inner], b[inner])
        say(f"judge region: {inner.sum()} inner cells of {mb.sum()} marked, identical")
        # start the next block from the full state
        for t_, src in zip((part.h, part.qx, part.qy), (full.h, full.qx, full.qy)):
            t_.copy_(src)
        part.rebind_fields()
        part.set_time(full.diag()["t"], full.diag()["step"])
    part.set_judge_region(None, 1)
