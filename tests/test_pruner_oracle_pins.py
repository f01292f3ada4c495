"""Pins of the pruner oracle against facts it does not compute itself:
library correlation, finite differences, closed forms, hand-worked cases and
a second formulation of the cell histograms."""
import math

import numpy as np
import pytest
from scipy.signal import correlate2d

import pd_synth
from oracle import pd_oracle as O
from oracle import pruner_oracle as P


def test_parameter_count_of_the_network():
    assert P.param_count() == 33505
    assert pd_synth.pruner_init().size == 33505
    layers, head = P.unpack(pd_synth.pruner_init())
    assert [w.shape for w, _ in layers] == [(32, 68, 3, 3), (32, 32, 3, 3), (16, 32, 3, 3)]
    assert head[0].shape == (16,)


def test_conv_equals_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(7, 9, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = P.conv3x3(x, w, b)
    for o in range(4):
        ref = b[o] + sum(correlate2d(x[:, :, c], w[o, c], mode="same", boundary="fill") for c in range(3))
        assert np.allclose(y[:, :, o], ref, atol=1e-12)


def test_conv_impulse_response():
    x = np.zeros((5, 6, 1))
    x[2, 3, 0] = 1.0
    w = np.arange(9, dtype=np.float64).reshape(1, 1, 3, 3)
    y = P.conv3x3(x, w, np.zeros(1))[:, :, 0]
    # y[p][q] = W[2 - p + 1][3 - q + 1] around the impulse, zero elsewhere
    for p in range(5):
        for q in range(6):
            u, v = 2 - p + 1, 3 - q + 1
            exp = w[0, 0, u, v] if 0 <= u < 3 and 0 <= v < 3 else 0.0
            assert y[p, q] == exp


def _loss(params, xs, labs, masks, pw, ch):
    zs = [P.forward(x, params, ch)[0] for x in xs]
    return P.bce_loss_grad(zs, labs, masks, pw)[0]


def test_backward_matches_central_differences():
    ch = (4, 3, 3, 2)
    rng = np.random.default_rng(1)
    params = rng.normal(0.0, 0.5, P.param_count(ch))
    xs = [rng.normal(size=(6, 5, 4)), rng.normal(size=(4, 7, 4))]
    labs = [(rng.random((6, 5)) < 0.3).astype(float), (rng.random((4, 7)) < 0.3).astype(float)]
    masks = [(rng.random((6, 5)) < 0.8).astype(float), np.ones((4, 7))]
    pw = 3.0
    zs, caches = zip(*[P.forward(x, params, ch) for x in xs])
    _, dz = P.bce_loss_grad(zs, labs, masks, pw)
    g = sum(P.backward(d, c, params, ch) for d, c in zip(dz, caches))
    h = 1e-6
    fd = np.zeros_like(params)
    for k in range(params.size):
        e = np.zeros_like(params)
        e[k] = h
        fd[k] = (_loss(params + e, xs, labs, masks, pw, ch) - _loss(params - e, xs, labs, masks, pw, ch)) / (2 * h)
    scale = np.abs(fd).max()
    assert np.abs(g - fd).max() <= 1e-6 * scale, np.abs(g - fd).max() / scale


def test_bce_closed_form_at_zero_logit():
    y = np.array([[1.0, 0.0, 1.0], [0.0, 0.0, 1.0]])
    m = np.array([[1.0, 1.0, 1.0], [1.0, 0.0, 1.0]])
    loss, (g,) = P.bce_loss_grad([np.zeros((2, 3))], [y], [m], 5.0)
    n_pos, n_neg = 3, 2
    assert math.isclose(loss, (5.0 * n_pos + n_neg) * math.log(2.0) / 5.0, rel_tol=1e-14)
    # dL/dz at z = 0: (1 - y) / 2 - pw * y / 2, over 5 masked cells
    assert np.allclose(g, m * ((1 - y) * 0.5 - 5.0 * y * 0.5) / 5.0, atol=1e-15)


def test_adam_first_steps_move_by_lr_times_sign():
    g = np.array([0.3, -2.0, 1e-3])
    p0 = np.array([1.0, 1.0, 1.0])
    p1, m, v = P.adam_step(p0, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p1, p0 - 0.01 * np.sign(g), rtol=0, atol=1e-7)
    # a constant gradient keeps bias-corrected moments at g and g^2
    p2, _, _ = P.adam_step(p1, g, m, v, 2, lr=0.01)
    assert np.allclose(p2, p1 - 0.01 * np.sign(g), rtol=0, atol=1e-7)
    p3, _, _ = P.adam_step(p0, np.zeros(3), np.zeros(3), np.zeros(3), 1)
    assert np.array_equal(p3, p0)


def test_cellmap_constant_image():
    img = np.full((32, 40), 77, np.uint8)
    cm = P.cellmap(img)
    assert cm.shape == (4, 5, 68)
    assert np.all(cm[:, :, :9] == 0.0)
    lbp = cm[:, :, 9:]
    assert np.all(lbp[:, :, 57] == 1.0) and lbp.sum() == 20.0  # code 255 -> bin 57, 64 / 64


def test_cellmap_horizontal_ramp_interior():
    a = 2
    img = np.tile((a * np.arange(64)).astype(np.uint8), (48, 1))
    hog = P.cell_hog_full(img)
    # dx = -2a, dy = 0: 180 deg folds to 0, half into bins 8 and 0; an interior
    # cell gathers spatial weights summing to 8 x 8
    for cy in range(1, 5):
        for cx in range(1, 7):
            exp = np.zeros(9)
            exp[0] = exp[8] = 64 * 2 * a * 0.5
            assert np.allclose(hog[cy, cx], exp, atol=1e-12)
    # top row: rows above the image do not exist, weights over y sum to 7
    assert np.allclose(hog[0, 3, [0, 8]], 7 * 8 * 2 * a * 0.5, atol=1e-12)
    v = P.cellmap(img)[2, 3, :9]
    assert math.isclose(v[0], 128 * a / 2 / math.sqrt(2 * (64 * a) ** 2 + 1e-6), rel_tol=1e-12)


def test_cell_hog_equals_scatter_from_pixel_cells():
    """Second formulation: every pixel of the grid scatters into the 3x3
    neighbouring cells with the per-axis weights of its offset in its cell."""
    img = pd_synth.frame(72, 56, 5)
    _, _, mag, ang = O.gradient(img)
    b0, b1, w0, w1 = O.orientation_votes(ang)
    hc, wc = 7, 9
    ref = np.zeros((hc, wc, 9))

    def sw(p, d):
        return max(0.0, 1.0 - abs(p + 0.5 - (8 * d + 4)) / 8.0)

    for y in range(8 * hc):
        for x in range(8 * wc):
            cy, cx, py, px = y // 8, x // 8, y % 8, x % 8
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    ty, tx = cy + dy, cx + dx
                    wgt = sw(py, dy) * sw(px, dx)
                    if wgt == 0.0 or not (0 <= ty < hc and 0 <= tx < wc):
                        continue
                    ref[ty, tx, b0[y, x]] += mag[y, x] * wgt * w0[y, x]
                    ref[ty, tx, b1[y, x]] += mag[y, x] * wgt * w1[y, x]
    assert np.allclose(P.cell_hog_full(img), ref, atol=1e-9)


def test_window_labels_and_topk():
    scores = np.array([[0.1, 2.0], [3.0, -1.0]])
    lab, mask = P.window_labels(18, 11, scores, 1.0)
    assert mask.sum() == 4 and mask[7, 3] == 1 and mask[8, 4] == 1 and mask[9, 3] == 0
    assert lab[7, 4] == 1 and lab[8, 3] == 1 and lab.sum() == 2
    z = [np.array([[0.5, 0.2], [0.9, 0.5]]), np.array([[0.5, -3.0]])]
    keep = P.keep_topk(z, 2)  # sorted: 0.9, 0.5, 0.5, 0.5, ... -> k-th = 0.5, ties kept
    assert [k.tolist() for k in keep] == [[[True, False], [True, True]], [[True, False]]]
    assert sum(k.sum() for k in P.keep_topk(z, 1)) == 1
    assert sum(k.sum() for k in P.keep_topk(z, 0)) == 0


def test_match_recall_cases():
    a, b = (0, 0, 100, 200), (300, 0, 400, 200)
    assert P.match_recall([], [a]) == 1.0
    assert P.match_recall([a, b], [a, b]) == 1.0
    assert P.match_recall([a, b], [a]) == 0.5
    # one pruned box cannot serve two plain boxes
    assert P.match_recall([a, (0, 0, 100, 190)], [a]) == 0.5
    # IoU exactly 0.5 matches: shift by a third of the width
    c = (0, 0, 90, 200)
    d = (30, 0, 120, 200)  # inter 60x200, union 120x200
    assert P.match_recall([c], [d]) == 1.0
    assert P.match_recall([c], [(31, 0, 121, 200)]) == 0.0
    # the larger-IoU box is taken first
    assert P.match_recall([a, (10, 0, 110, 200)], [(5, 0, 105, 200), a]) == 1.0
