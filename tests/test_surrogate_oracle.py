"""Pins of the FP64 surrogate oracle: convolution indexing and padding by
closed forms, backward by central finite differences, Adam's first step."""
import numpy as np
import pytest

from oracle import surrogate_oracle as S


def test_identity_and_shift_kernels():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 6, 7, 4))
    w = np.zeros((4, 3, 3, 4))
    for c in range(4):
        w[c, 1, 1, c] = 1.0
    assert np.array_equal(S.conv3x3(x, w, np.zeros(4)), x)
    # a single tap at (dy, dx) = (0, 2) reads x[i-1, j+1]
    w = np.zeros((4, 3, 3, 4))
    for c in range(4):
        w[c, 0, 2, c] = 1.0
    y = S.conv3x3(x, w, np.zeros(4))
    exp = np.zeros_like(x)
    exp[:, 1:, :-1, :] = x[:, :-1, 1:, :]
    assert np.array_equal(y, exp)


def test_box_kernel_counts_neighbours():
    x = np.full((1, 5, 6, 1), 2.0)
    y = S.conv3x3(x, np.ones((1, 3, 3, 1)), np.array([0.5]))[0, ..., 0]
    assert y[2, 3] == 9 * 2 + 0.5 and y[0, 3] == 6 * 2 + 0.5 and y[0, 0] == 4 * 2 + 0.5


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    params = S.init_params(3)
    # non-zero biases so every ReLU pattern is exercised
    params = [(w, rng.normal(0, 0.1, size=b.shape)) for w, b in params]
    x = rng.normal(size=(2, 4, 5, S.CIN0))
    x[..., 5:] = 0.0
    target = rng.normal(size=(2, 4, 5, 3))
    loss, grads = S.loss_and_grads(params, x, target)
    eps = 1e-6
    for li, (w, b) in enumerate(params):
        dw, db = grads[li]
        idx = [tuple(rng.integers(0, n) for n in w.shape) for _ in range(12)]
        for ix in idx:
            wp = [(p.copy(), q.copy()) for p, q in params]
            wm = [(p.copy(), q.copy()) for p, q in params]
            wp[li][0][ix] += eps
            wm[li][0][ix] -= eps
            fd = (S.loss_and_grads(wp, x, target)[0] - S.loss_and_grads(wm, x, target)[0]) / (2 * eps)
            assert fd == pytest.approx(dw[ix], rel=1e-5, abs=1e-9), (li, ix)
        for o in rng.integers(0, len(b), 4):
            bp = [(p.copy(), q.copy()) for p, q in params]
            bm = [(p.copy(), q.copy()) for p, q in params]
            bp[li][1][o] += eps
            bm[li][1][o] -= eps
            fd = (S.loss_and_grads(bp, x, target)[0] - S.loss_and_grads(bm, x, target)[0]) / (2 * eps)
            assert fd == pytest.approx(db[o], rel=1e-5, abs=1e-9), (li, o)


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = S.adam_update(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-12)


def test_pack_and_apply():
    rng = np.random.default_rng(2)
    h, hu, hv, z, occ = (rng.uniform(0, 1, (3, 4)) for _ in range(5))
    x = S.pack_input(h, hu, hv, z, occ)
    assert np.allclose(x[..., 3], z / 3.0) and np.all(x[..., 5:] == 0)
    hn, qun, qvn = S.apply_output(h, hu, hv, np.zeros((3, 4, 3)))
    assert np.array_equal(hn, h) and np.array_equal(qun, hu) and np.array_equal(qvn, hv)


def test_apply_output_zeroes_discharge_where_dry():
    h = np.array([[0.5, 0.02]])
    hu = np.array([[0.1, 0.3]])
    hv = np.array([[-0.2, 0.1]])
    y = np.zeros((1, 2, 3))
    y[0, 1, 0] = -1.0                      # 0.02 - 0.05 -> dry
    hn, qx, qy = S.apply_output(h, hu, hv, y)
    assert hn[0, 1] == 0.0 and qx[0, 1] == 0.0 and qy[0, 1] == 0.0
    assert hn[0, 0] == 0.5 and qx[0, 0] == 0.1 and qy[0, 0] == -0.2


def test_make_target_inverts_apply_output():
    rng = np.random.default_rng(4)
    h0, hu0, hv0 = (rng.uniform(0.1, 1, (5, 6)) for _ in range(3))
    h1, hu1, hv1 = (a + rng.uniform(-0.05, 0.05, a.shape) for a in (h0, hu0, hv0))
    t = S.make_target(h0, hu0, hv0, h1, hu1, hv1)
    for got, want in zip(S.apply_output(h0, hu0, hv0, t), (h1, hu1, hv1)):
        assert np.allclose(got, want, rtol=0, atol=1e-14)


def test_hazard_class_thresholds_table1():
    thr = (0.75, 1.5, 2.5)
    # HR = (|u| + 0.5) h: h = 1 m still water -> 0.5 (low); u = 0.5 -> 1.0 (medium);
    # u = 1.5 -> 2.0 (high); u = 2.0 -> 2.5 (highest: the bound is exclusive)
    h = np.ones(5, np.float32)
    q = np.array([0.0, 0.5, 1.5, 2.0, -2.0], np.float32)
    assert list(S.hazard_class32(h, q, 0 * q, 1e-5, thr)) == [1, 2, 3, 4, 4]
    assert list(S.hazard_class32(h, 0 * q, q, 1e-5, thr)) == [1, 2, 3, 4, 4]
    assert S.hazard_class32(np.float32(1e-6), np.float32(5.0), np.float32(0), 1e-5, thr) == 0


def test_judge_counts_by_hand():
    thr = (0.75, 1.5, 2.5)
    nx, ny, dx, dy = 4, 3, 2.0, 2.0
    hb = np.full((ny, nx), 0.5, np.float32)
    qb = np.zeros((ny, nx), np.float32)
    ha = hb.copy()
    ha[0, 0] = 0.505                       # within 1 cm, same class: fine
    ha[1, 2] = 0.52                        # 2 cm off: bad
    qa = qb.copy()
    qa[2, 3] = 0.6                         # same depth, HR 0.25 -> 0.85: class changes
    # agents: one per altered cell, one exited on the bad cell, one outside (clamped)
    x = np.array([1.0, 5.0, 7.9, 5.5, -3.0, 100.0], np.float32)
    y = np.array([1.0, 3.0, 5.0, 3.5, 1.0, 100.0], np.float32)
    st = np.array([0, 0, 0, 1, 0, 0], np.uint8)
    n, dmax, judged = S.judge(x, y, st, nx, ny, dx, dy, (ha, qa, qb), (hb, qb, qb), 0.01, 1e-5, thr)
    # bad: agent 1 (cell (2,1)), agent 2 (cell (3,2)), agent 5 (clamped to (3,2))
    assert n == 3 and judged == 5
    assert dmax == np.float32(0.52) - np.float32(0.5)
    same = S.judge(x, y, st, nx, ny, dx, dy, (hb, qb, qb), (hb, qb, qb), 0.01, 1e-5, thr)
    assert same == (0, 0.0, 5)
    # every third agent: agent 0 (fine) and agent 3 (exited)
    assert S.judge(x, y, st, nx, ny, dx, dy, (ha, qa, qb), (hb, qb, qb), 0.01, 1e-5, thr, stride=3) == (
        0, float(np.float32(0.505) - np.float32(0.5)), 1)
    # the sample (agent 0) plus the people near a class boundary of a selection
    # state: cell (2,1) at HR 0.5 x 1.45 = 0.725, 0.025 below the first
    # threshold; cell (3,2) dry
    hs = np.full((ny, nx), 0.5, np.float32)
    hs[1, 2] = 1.45
    hs[2, 3] = 0.0
    sel = (hs, qb, qb)
    r = S.judge(x, y, st, nx, ny, dx, dy, (ha, qa, qb), (hb, qb, qb), 0.01, 1e-5, thr, stride=1000, select=sel,
                hr_margin=0.05)
    assert r[0] == 3 and r[2] == 4            # agents 0, 1, 2, 5 judged; 1, 2, 5 off
    r = S.judge(x, y, st, nx, ny, dx, dy, (ha, qa, qb), (hb, qb, qb), 0.01, 1e-5, thr, stride=1000, select=sel,
                hr_margin=0.02)
    assert r[0] == 2 and r[2] == 3            # 0.025 away is outside a 0.02 margin: agent 1 not judged
    # a depth margin makes the 0.5 m cells "near dry" as well (agents 0, 4 and, dry,
    # 2 and 5), but not the 1.45 m cell of agent 1
    r = S.judge(x, y, st, nx, ny, dx, dy, (ha, qa, qb), (hb, qb, qb), 0.01, 1e-5, thr, stride=1000, select=sel,
                h_margin=0.6)
    assert r[0] == 2 and r[2] == 4


def test_bf16_round_ties_to_even_and_matches_library():
    one = 1.0
    assert S.bf16_round(one + 2.0 ** -8) == 1.0                    # tie -> even (down)
    assert S.bf16_round(one + 3 * 2.0 ** -8) == one + 2.0 ** -6    # tie -> even (up)
    assert S.bf16_round(one + 2.0 ** -8 + 2.0 ** -20) == one + 2.0 ** -7
    assert S.bf16_round(-3.0) == -3.0 and S.bf16_round(0.0) == 0.0
    import torch
    v = np.random.default_rng(6).normal(0, 10, 10000)
    lib = torch.tensor(v, dtype=torch.float32).bfloat16().double().numpy()
    assert np.array_equal(S.bf16_round(v), lib)


def test_bf16_rounding_points_change_only_rounding():
    """The BF16 network stays within BF16 rounding of the FP64 one: output
    relative error a few BF16 units, last-layer gradients close."""
    rng = np.random.default_rng(8)
    params = [(S.bf16_round(w), b) for w, b in S.init_params(8)]
    x = np.zeros((1, 6, 7, S.CIN0))
    x[..., :5] = S.bf16_round(rng.uniform(-1, 1, (1, 6, 7, 5)))
    t = rng.normal(0, 0.5, (1, 6, 7, 3))
    y0, _, _ = S.forward(params, x)
    y1, _, _ = S.forward(params, x, bf16=True)
    assert 0 < np.linalg.norm(y1 - y0) / np.linalg.norm(y0) < 2e-2
    _, g0 = S.loss_and_grads(params, x, t)
    _, g1 = S.loss_and_grads(params, x, t, bf16=True)
    dw0, dw1 = g0[-1][0], g1[-1][0]
    assert np.linalg.norm(dw1 - dw0) / np.linalg.norm(dw0) < 2e-2


def test_apply_output_keeps_dry_cells_dry_below_snap():
    h = np.array([[0.0, 0.0, 5e-6, 0.3]])
    z = np.zeros_like(h)
    y = np.zeros((1, 4, 3))
    y[0, :, 0] = [0.5e-3 / 0.05, 2e-3 / 0.05, 0.5e-3 / 0.05, -0.299 / 0.05]
    y[0, :, 1] = 0.2
    hn, qx, qy = S.apply_output(h, z, z, y)
    # 0.5 mm on a dry cell: stays dry; 2 mm: wets; 1 mm left on a wet cell: kept
    assert hn[0, 0] == 0.0 and qx[0, 0] == 0.0
    assert abs(hn[0, 1] - 2e-3) < 1e-15 and qx[0, 1] == 0.2 * 0.05
    assert hn[0, 2] == 0.0
    assert abs(hn[0, 3] - 1e-3) < 1e-12


def test_pack_input_inflow_channel_on_each_side():
    ny, nx = 5, 7
    zero = np.zeros((ny, nx))
    for side, where in ((2, (0, slice(2, 5))), (3, (ny - 1, slice(2, 5))), (0, (slice(2, 5), 0)),
                        (1, (slice(2, 5), nx - 1))):
        x = S.pack_input(zero, zero, zero, zero, zero, inflow=(side, 2, 5, 0.3))
        want = np.zeros((ny, nx))
        want[where] = 0.3
        assert np.array_equal(x[..., 5], want)
    assert np.all(S.pack_input(zero, zero, zero, zero, zero, inflow=(-1, 0, 0, 1.0))[..., 5] == 0)
