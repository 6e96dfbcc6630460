"""GPU parity of the BF16 MFMA surrogate kernels against the FP64 oracle.

The GPU rounds weights and activations to BF16 and accumulates in FP32; the
oracle gets the same BF16-rounded weights and inputs and computes in FP64.
Bars: forward relative L2 error <= 2e-2; per-tensor gradients cosine >= 0.999
and relative L2 error <= 2e-2."""
import numpy as np
import pytest
import torch

from oracle import surrogate_oracle as S
from paper_1908_05232_amd import fps
from tests.gpu_util import say

pytestmark = pytest.mark.gpu
COUT_GPU = [64, 64, 64, 64, 16]


def bf16_round(a):
    return torch.tensor(np.asarray(a, np.float32)).bfloat16().float().numpy().astype(np.float64)


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
    yo, _, _ = S.forward(params, x)
    err = rel_l2(y[..., :3], yo)
    say(f"surrogate forward rel L2 {err:.2e}")
    assert err <= 2e-2
    assert np.all(y[..., 3] == 0.0)


def test_gradients_match_oracle():
    params, x, target = make_case(2, 2, 16, 64)
    sur = fps.Surrogate(2, 16, 64)
    p, xt, tt = to_dev(params, x, target)
    sur.set_params(p)
    loss, g = sur.gradients(xt, tt)
    lo, go = S.loss_and_grads(params, x, target)
    assert float(loss.item()) == pytest.approx(lo, rel=2e-2)
    gg = unpack(g.cpu().numpy().astype(np.float64), params)
    for li, ((dw, db), (dwo, dbo)) in enumerate(zip(gg, go)):
        if li == 0:
            dw, dwo = dw[..., :5], dwo[..., :5]       # zero input channels carry no gradient
        c, e = cosine(dw, dwo), rel_l2(dw, dwo)
        cb, eb = cosine(db, dbo), rel_l2(db, dbo)
        say(f"layer {li + 1}: dW cos {c:.6f} rel {e:.2e}; db cos {cb:.6f} rel {eb:.2e}")
        assert c >= 0.999 and e <= 2e-2 and cb >= 0.999 and eb <= 2e-2


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
    x = fps.sur_pack(*dev).float().cpu().numpy()
    xo = S.pack_input(*(a.astype(np.float64) for a in (h, hu, hv, z, occ)))
    xr = bf16_round(xo)
    keep = [0, 1, 2, 4] + list(range(5, 16))
    assert np.array_equal(x[..., keep], xr[..., keep])
    assert np.allclose(x[..., 3], xr[..., 3], rtol=2.0 ** -7, atol=0)   # z / 3: one bf16 ulp
    x0 = fps.sur_pack(*dev[:4]).float().cpu().numpy()       # no occupancy
    assert np.all(x0[..., 4] == 0) and np.array_equal(x0[..., :4], x[..., :4])
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
    want = S.judge(x, y, st, nx, ny, dx, dy, a, b, 0.01, 1e-5, (0.75, 1.5, 2.5))
    dv = lambda arr: torch.tensor(arr).cuda()
    out = fps.sur_judge(dv(x), dv(y), dv(st), nx, ny, dx, dy, tuple(map(dv, a)), tuple(map(dv, b)))
    got = fps.judge_result(out)
    say(f"judge: {got} oracle {want}")
    assert got[0] == want[0] and got[1] == want[1] and want[0] > 0
    # no agents -> (0, 0); identical states -> (0, 0)
    out0 = fps.sur_judge(dv(x[:0]), dv(y[:0]), dv(st[:0]), nx, ny, dx, dy, tuple(map(dv, a)),
                         tuple(map(dv, b)))
    assert fps.judge_result(out0) == (0, 0.0)
    same = fps.sur_judge(dv(x), dv(y), dv(st), nx, ny, dx, dy, tuple(map(dv, b)), tuple(map(dv, b)))
    assert fps.judge_result(same) == (0, 0.0)
