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
