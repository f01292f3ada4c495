"""Pins of the FP64 oracle against facts fixed by the paper and by the
mathematics (hand-worked values, closed forms, invariants, special cases
that reduce to textbook routines, brute force on tiny inputs).  CPU only."""
import math
import os

import numpy as np
import pytest

import pd_synth
from oracle import pd_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- pyramid --

def test_level_sizes_road_frame():
    # 1242x375 at scale 11/10: twelve levels down to 435x131 (the next,
    # 395x119, is shorter than the 128-pixel window).
    sizes = O.level_sizes(1242, 375)
    assert sizes == [(1242, 375), (1129, 340), (1026, 309), (933, 281), (848, 256),
                     (771, 232), (701, 211), (637, 192), (579, 174), (526, 159),
                     (478, 144), (435, 131)]
    wins = [O.window_grid(w, h) for (w, h) in sizes]
    assert [a * b for a, b in wins] == [4588, 3618, 2783, 2180, 1683, 1246, 880, 648,
                                       390, 232, 156, 47]
    assert sum(a * b for a, b in wins) == 18451


def test_level_sizes_small_config():
    sizes = O.level_sizes(320, 240, 6, 5, max_levels=3)
    assert sizes == [(320, 240), (266, 200), (222, 166)]
    assert sum(a * b for a, b in (O.window_grid(w, h) for w, h in sizes)) == 495 + 260 + 100


def test_level_sizes_too_small():
    assert O.level_sizes(63, 500) == []
    assert O.level_sizes(500, 127) == []
    assert O.level_sizes(64, 128) == [(64, 128)]


def test_resize_level0_is_identity():
    img = pd_synth.frame(97, 61, 3)
    assert np.array_equal(O.resize(img, 97, 61), img)


def test_resize_constant_stays_constant():
    for v in (0, 1, 77, 254, 255):
        img = np.full((131, 257), v, np.uint8)
        assert np.all(O.resize(img, 190, 77) == v)


def test_resize_hand_worked_row():
    # Q8 source coordinate ((2x+1) W0 - Wk) * 128 // Wk, worked by hand.
    row = np.array([[0, 100, 200, 255]], np.uint8)
    x0, fx, _ = O._axis_q8(4, 3)
    assert list(zip(x0.tolist(), fx.tolist())) == [(0, 42), (1, 128), (2, 213)]
    assert O.resize(row, 3, 1).tolist() == [[16, 150, 246]]
    # 227.5 rounds half up to 228
    assert O.resize(row, 2, 1).tolist() == [[50, 228]]
    x0, fx, _ = O._axis_q8(320, 266)
    assert (int(x0[0]), int(fx[0])) == (0, 25)


def test_resize_halving_is_2x2_mean_rounded_half_up():
    # For W0 = 2 Wk the source coordinate is exactly between two pixels, so
    # bilinear resize is the 2x2 box mean, rounded half up.
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, size=(40, 66), dtype=np.uint8)
    out = O.resize(img, 33, 20)
    s = img.astype(np.int64).reshape(20, 2, 33, 2).sum(axis=(1, 3))
    assert np.array_equal(out.astype(np.int64), (s + 2) // 4)


def test_resize_matches_float_bilinear_at_q8_coordinates():
    # Independent float evaluation at the same Q8 sample points.
    rng = np.random.default_rng(6)
    img = rng.integers(0, 256, size=(37, 53), dtype=np.uint8)
    wk, hk = 41, 29
    out = O.resize(img, wk, hk)
    for y in range(hk):
        sy = (((2 * y + 1) * 37 - hk) * 128) // hk / 256.0
        for x in range(wk):
            sx = (((2 * x + 1) * 53 - wk) * 128) // wk / 256.0
            ya, xa = int(math.floor(sy)), int(math.floor(sx))
            yb, xb = min(ya + 1, 36), min(xa + 1, 52)
            ty, tx = sy - ya, sx - xa
            v = ((1 - ty) * ((1 - tx) * img[ya, xa] + tx * img[ya, xb])
                 + ty * ((1 - tx) * img[yb, xa] + tx * img[yb, xb]))
            assert out[y, x] == math.floor(v + 0.5)


# -------------------------------------------------------------------- LBP --

def _read_patches():
    rows = []
    for line in open(os.path.join(GOLDEN, "lbp_patches.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        vals, code, b = line.split("|")
        rows.append((np.array([int(v) for v in vals.split()], np.uint8).reshape(3, 3),
                     int(code), int(b)))
    return rows


def test_uniform_table_matches_hand_list():
    line = [l for l in open(os.path.join(GOLDEN, "lbp_uniform_ranks.txt")) if not l.startswith("#")]
    hand = [int(v) for v in " ".join(line).split()]
    table = O.uniform_bin_table()
    assert len(hand) == 58 == P_UNIFORM(8)
    assert [c for c in range(256) if table[c] < 58] == hand
    assert [int(table[c]) for c in hand] == list(range(58))
    assert table[5] == 58 and table[228] == 58


def P_UNIFORM(p):
    # number of uniform patterns with p neighbours: p (p - 1) + 2
    return p * (p - 1) + 2


def test_lbp_hand_worked_patches():
    table = O.uniform_bin_table()
    for patch, code, b in _read_patches():
        got = O.lbp_codes(patch)[1, 1]
        assert got == code, (patch, got, code)
        assert table[got] == b


def test_lbp_constant_image():
    img = np.full((24, 40), 123, np.uint8)
    assert np.all(O.lbp_codes(img) == 255)
    h = O.lbp_cell_histograms(img)
    assert h.shape == (3, 5, 59)
    assert np.all(h[..., 57] == 64) and h.sum() == 64 * 15


def test_lbp_cell_sums_and_ragged_edge():
    img = pd_synth.frame(77, 45, 9)   # 9x5 whole cells, 5 and 5 spare pixels
    h = O.lbp_cell_histograms(img)
    assert h.shape == (5, 9, 59)
    assert np.all(h.sum(axis=-1) == 64)


def test_lbp_edge_clamp_corner():
    # top-left corner pixel: TL, T, TR, L, BL clamp onto the row/column itself
    img = np.array([[5, 9], [9, 9]], np.uint8)
    # centre 5; TL->5 (>=), T->5, TR->9, R->9, BR->9, B->9, BL->9 (clamped to
    # column 0 of row 1), L->5: every neighbour >= 5 -> 255
    assert O.lbp_codes(img)[0, 0] == 255
    img = np.array([[9, 1], [1, 1]], np.uint8)
    # centre 9; clamped copies of itself (TL, T, L) give 1 -> bits 0, 1, 7;
    # TR (clamped to row 0: 1), R, BR, B, BL are 1 < 9 -> 0
    assert O.lbp_codes(img)[0, 0] == 1 + 2 + 128


# ---------------------------------------------------------------- gradient --

def _grad_case(left, right, up, down):
    img = np.zeros((3, 3), np.uint8)
    img[1, 0], img[1, 2], img[0, 1], img[2, 1] = left, right, up, down
    dx, dy, m, a = O.gradient(img)
    return dx[1, 1], dy[1, 1], m[1, 1], a[1, 1]


def test_gradient_hand_worked():
    dx, dy, m, a = _grad_case(10, 40, 7, 7)      # dx = 10 - 40 = -30
    assert (dx, dy, m, a) == (-30, 0, 30, 0.0)   # 180 deg folds to 0
    b0, b1, w0, w1 = O.orientation_votes(a)
    assert (b0, b1, w0, w1) == (8, 0, 0.5, 0.5)
    dx, dy, m, a = _grad_case(5, 5, 0, 30)       # dy = 0 - 30, -90 -> 90
    assert (dx, dy, m) == (0, -30, 30) and abs(a - 90.0) < 1e-12
    b0, b1, w0, w1 = O.orientation_votes(a)
    assert (b0, w0) == (4, 1.0) and w1 == 0.0
    dx, dy, m, a = _grad_case(40, 20, 40, 20)    # (20, 20) -> 45 deg
    assert abs(m - 20 * math.sqrt(2)) < 1e-12 and abs(a - 45.0) < 1e-12
    b0, b1, w0, w1 = O.orientation_votes(a)
    assert (b0, b1) == (1, 2) and abs(w0 - 0.25) < 1e-12 and abs(w1 - 0.75) < 1e-12
    dx, dy, m, a = _grad_case(20, 40, 40, 20)    # (-20, 20) -> 135 deg
    assert abs(a - 135.0) < 1e-12
    b0, b1, w0, w1 = O.orientation_votes(a)
    assert (b0, b1) == (6, 7) and abs(w0 - 0.75) < 1e-12 and abs(w1 - 0.25) < 1e-12


def test_gradient_constant_image_has_zero_magnitude():
    _, _, m, _ = O.gradient(np.full((16, 16), 200, np.uint8))
    assert np.all(m == 0)


def test_gradient_edge_clamp():
    img = np.arange(5, dtype=np.uint8)[None, :].repeat(3, 0) * 10
    dx, dy, _, _ = O.gradient(img)
    assert dx[1].tolist() == [-10, -20, -20, -20, -10]
    assert np.all(dy == 0)


# ------------------------------------------------------------------- HOG --

def test_spatial_weights_closed_form():
    w = [O.spatial_weight(p, 0) for p in range(16)]
    assert w[:8] == [0.5625, 0.6875, 0.8125, 0.9375, 0.9375, 0.8125, 0.6875, 0.5625]
    assert w[8:] == [0.4375, 0.3125, 0.1875, 0.0625, 0, 0, 0, 0]
    assert sum(w) == 7.0
    assert [O.spatial_weight(p, 1) for p in range(16)] == w[::-1]


def test_hog_single_impulse_hand_worked():
    # One pixel with M = 1, theta = 45 deg (bins 1 and 2 at 0.25 / 0.75) at
    # (y, x) = (12, 5): it lies in blocks (0, 0) (offset 12, 5) and (1, 0)
    # (offset 4, 5).  Weights worked by hand from the cell-centre distances.
    mag = np.zeros((32, 24))
    ang = np.zeros((32, 24))
    mag[12, 5], ang[12, 5] = 1.0, 45.0
    h = O.hog_block_histograms(mag, ang)
    assert h.shape == (3, 2, 36)
    exp = np.zeros((3, 2, 36))
    # block (0,0): wy = (0, 0.9375), wx = (0.8125, 0.1875)
    for (r, c, w) in [(1, 0, 0.9375 * 0.8125), (1, 1, 0.9375 * 0.1875)]:
        exp[0, 0, (r * 2 + c) * 9 + 1] = 0.25 * w
        exp[0, 0, (r * 2 + c) * 9 + 2] = 0.75 * w
    # block (1,0): wy = (0.9375, 0.0625), wx = (0.8125, 0.1875)
    for (r, c, w) in [(0, 0, 0.9375 * 0.8125), (0, 1, 0.9375 * 0.1875),
                      (1, 0, 0.0625 * 0.8125), (1, 1, 0.0625 * 0.1875)]:
        exp[1, 0, (r * 2 + c) * 9 + 1] = 0.25 * w
        exp[1, 0, (r * 2 + c) * 9 + 2] = 0.75 * w
    assert np.array_equal(h, exp)


def test_hog_pixel_votes_two_four_or_eight_bins():
    # Section 4.3: each pixel falls in two, four or eight bins of a block.
    counts = set()
    for py in range(16):
        for px in range(16):
            for ang in (45.0, 40.0):   # 40 deg sits on a bin centre: 1 bin
                mag = np.zeros((16, 16))
                a = np.zeros((16, 16))
                mag[py, px], a[py, px] = 1.0, ang
                counts.add((ang, int(np.count_nonzero(O.hog_block_histograms(mag, a)))))
    assert {c for (a, c) in counts if a == 45.0} == {2, 4, 8}


def test_hog_horizontal_ramp_closed_form():
    img = np.tile(np.arange(160, dtype=np.uint8), (64, 1))  # I = x
    f = O.hog_features(img)
    interior = f[1:-1, 1:-1]
    exp = 0.2 / math.sqrt(8 * 0.04 + 1e-6)      # 8 equal entries, clipped
    nz = interior[..., [0, 8, 9, 17, 18, 26, 27, 35]]
    assert np.allclose(nz, exp, rtol=0, atol=1e-12)
    mask = np.ones(36, bool)
    mask[[0, 8, 9, 17, 18, 26, 27, 35]] = False
    assert np.all(interior[..., mask] == 0)


def test_hog_vertical_ramp_closed_form():
    img = np.tile(np.arange(96, dtype=np.uint8)[:, None], (1, 48))  # I = y
    f = O.hog_features(img)
    interior = f[1:-1, 1:-1]
    exp = 0.2 / math.sqrt(4 * 0.04 + 1e-6)
    assert abs(exp - 0.49999844) < 1e-8
    assert np.allclose(interior[..., [4, 13, 22, 31]], exp, rtol=0, atol=1e-12)
    assert np.count_nonzero(interior) == 4 * interior.shape[0] * interior.shape[1]


def test_hog_constant_image_is_zero():
    assert np.all(O.hog_features(np.full((40, 48), 90, np.uint8)) == 0)


def test_l2hys_bounds_and_clip():
    f = O.hog_features(pd_synth.frame(96, 80, 11))
    n = np.sqrt((f * f).sum(-1))
    assert np.all(n <= 1.0) and n.max() > 0.99
    assert f.max() <= 0.2 / math.sqrt(0.04 * 1 + 1e-6) + 1e-12
    v = np.array([3.0, 4.0, 0.0])
    # hand: 3/5.0000001, 4/5.0000001 -> 0.6, 0.8 -> clip 0.2, 0.2 -> 0.7071
    out = O.l2hys(v)
    assert np.allclose(out, [0.2 / math.sqrt(0.08 + 1e-6)] * 2 + [0.0], atol=1e-12)


def _hog_cell_partials(mag, ang):
    """Second formulation written for this test: each pixel votes once into
    its own cell's partial histograms towards the 3x3 neighbouring cell
    centres; a block sums the partials of its four cells that point at each
    of its four cell centres."""
    h, w = mag.shape
    hc, wc = h // 8, w // 8
    A = np.zeros((hc, wc, 3, 3, 9))
    for y in range(hc * 8):
        for x in range(wc * 8):
            m = mag[y, x]
            if m == 0:
                continue
            b0, b1, w0, w1 = O.orientation_votes(ang[y, x])
            cy, cx = y // 8, x // 8
            for dy in (-1, 0, 1):
                wy = max(0.0, 1.0 - abs(y + 0.5 - (8 * (cy + dy) + 4)) / 8)
                for dx in (-1, 0, 1):
                    wx = max(0.0, 1.0 - abs(x + 0.5 - (8 * (cx + dx) + 4)) / 8)
                    A[cy, cx, dy + 1, dx + 1, b0] += m * wy * wx * w0
                    A[cy, cx, dy + 1, dx + 1, b1] += m * wy * wx * w1
    out = np.zeros((hc - 1, wc - 1, 36))
    for by in range(hc - 1):
        for bx in range(wc - 1):
            for r in (0, 1):
                for c in (0, 1):
                    for sy in (by, by + 1):
                        for sx in (bx, bx + 1):
                            out[by, bx, (r * 2 + c) * 9:(r * 2 + c) * 9 + 9] += \
                                A[sy, sx, by + r - sy + 1, bx + c - sx + 1]
    return out


def test_hog_direct_equals_cell_partials():
    img = pd_synth.frame(57, 42, 21)
    _, _, m, a = O.gradient(img)
    direct = O.hog_block_histograms(m, a)
    other = _hog_cell_partials(m, a)
    assert direct.shape == other.shape == (4, 6, 36)
    assert np.allclose(direct, other, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- scoring --

def _features(seed=4, w=96, h=160):
    img = pd_synth.frame(w, h, seed)
    return O.level_features(img)


def test_window_grid_counts():
    assert O.window_grid(64, 128) == (1, 1)
    assert O.window_grid(71, 135) == (1, 1)
    assert O.window_grid(72, 136) == (2, 2)
    assert O.window_grid(1242, 375) == (31, 148)


def test_scores_brute_force_vs_correlation():
    hog, cells = _features()
    w = pd_synth.svm_weights(2)
    b = np.array([0.25, -1.5], np.float32)
    s = O.window_scores(hog, cells, w, b)
    ny, nx = s.shape[1:]
    wh = w[:, :O.HOG_DIM].astype(np.float64).reshape(2, 15, 7, 36)
    wl = w[:, O.HOG_DIM:].astype(np.float64).reshape(2, 16, 8, 59)
    corr = np.zeros_like(s)
    for a in range(15):
        for bb in range(7):
            corr += np.einsum("yxc,mc->myx", hog[a:a + ny, bb:bb + nx], wh[:, a, bb])
    for a in range(16):
        for bb in range(8):
            corr += np.einsum("yxc,mc->myx", cells[a:a + ny, bb:bb + nx].astype(np.float64), wl[:, a, bb])
    corr += b.astype(np.float64)[:, None, None]
    assert np.allclose(s, corr, rtol=1e-12, atol=1e-12)


def test_indicator_weight_is_a_gather():
    hog, cells = _features()
    w = np.zeros((2, O.FEATURE_DIM), np.float32)
    w[0, (3 * 7 + 5) * 36 + 17] = 1.0            # HOG block (3, 5), entry 17
    w[1, O.HOG_DIM + (11 * 8 + 2) * 59 + 58] = 1.0  # LBP cell (11, 2), bin 58
    s = O.window_scores(hog, cells, w, np.zeros(2))
    ny, nx = s.shape[1:]
    for i in range(ny):
        for j in range(nx):
            assert s[0, i, j] == hog[i + 3, j + 5, 17]
            assert s[1, i, j] == cells[i + 11, j + 2, 58]


def test_window_vector_layout():
    hog, cells = _features()
    v = O.window_vector(hog, cells, 1, 2)
    assert v.size == 11332
    assert v[0] == hog[1, 2, 0] and v[35] == hog[1, 2, 35] and v[36] == hog[1, 3, 0]
    assert v[7 * 36] == hog[2, 2, 0]
    assert v[3780] == cells[1, 2, 0] and v[3780 + 59] == cells[1, 3, 0]
    assert v[3780 + 8 * 59] == cells[2, 2, 0]


# ------------------------------------------------------- threshold / NMS --

def test_threshold_exactly_k_above():
    rng = np.random.default_rng(3)
    for n in (1, 2, 99, 100, 101, 855, 18451):
        s = rng.normal(size=n)
        t = O.threshold_99(s)
        assert np.count_nonzero(s > t) == math.ceil(0.01 * n)


def test_box_level0_and_scaled():
    assert O.window_box_q8(1242, 375, 1242, 375, 2, 3) == (24 * 256, 16 * 256, 88 * 256, 144 * 256)
    # level 11 (435x131) of 1242x375, window (0, 0):
    # x1 = floor(20348928 / 435) = 46779, y1 = floor(12288000 / 131) = 93801
    assert O.window_box_q8(1242, 375, 435, 131, 0, 0) == (0, 0, 46779, 93801)


def _read_nms():
    cases = []
    for line in open(os.path.join(GOLDEN, "nms_cases.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        name, boxes, kept = line.split("|")
        cands = []
        for q in boxes.split(";"):
            s, lv, i, j = q.split()
            cands.append({"score": float(s), "level": int(lv), "i": int(i), "j": int(j),
                          "box": O.window_box_q8(1242, 375, 1242, 375, int(i), int(j)), "id": len(cands)})
        cases.append((name.strip(), cands, [int(k) for k in kept.split()]))
    return cases


@pytest.mark.parametrize("case", _read_nms(), ids=lambda c: c[0])
def test_nms_hand_cases(case):
    name, cands, kept = case
    assert [c["id"] for c in O.nms(cands)] == kept


def test_select_top_hand_case():
    c = [{"score": 1.0, "level": 0, "i": 5, "j": 0}, {"score": 2.0, "level": 1, "i": 0, "j": 0},
         {"score": 1.0, "level": 0, "i": 2, "j": 9}, {"score": 1.0, "level": 1, "i": 0, "j": 0},
         {"score": 0.5, "level": 0, "i": 0, "j": 0}]
    got = [(d["score"], d["level"], d["i"], d["j"]) for d in O.select_top(c, 3)]
    assert got == [(2.0, 1, 0, 0), (1.0, 0, 2, 9), (1.0, 0, 5, 0)]
    assert O.select_top(c, 10) == O.select_top(c, 5) and len(O.select_top(c, 0)) == 0


def test_select_top_by_rank_counting():
    """A candidate is selected iff fewer than `limit` others precede it in the
    strict NMS order (counted pairwise, no sort)."""
    rng = np.random.default_rng(11)
    for n, limit in ((30, 7), (64, 64), (50, 1)):
        c = [{"score": float(rng.integers(0, 5)), "level": int(rng.integers(0, 3)), "i": int(q), "j": int(rng.integers(0, 4))}
             for q in range(n)]

        def before(a, b):
            return a["score"] > b["score"] or (a["score"] == b["score"] and
                                               (a["level"], a["i"], a["j"]) < (b["level"], b["i"], b["j"]))
        exp = {id(d) for d in c if sum(before(e, d) for e in c) < limit}
        assert {id(d) for d in O.select_top(c, limit)} == exp


def test_max_over_models_ties_lowest():
    s = np.array([[[1.0, 2.0]], [[1.0, 3.0]]])
    v, m = O.max_over_models(s)
    assert v.tolist() == [[1.0, 3.0]] and m.tolist() == [[0, 1]]


def test_detect_small_frame_consistency():
    img = pd_synth.frame(320, 240, 1000)
    w = pd_synth.svm_weights(1)
    levels, thr, cands, kept = O.detect(img, w, pd_synth.svm_bias(1), scale_num=6, scale_den=5, max_levels=3)
    assert [lv["size"] for lv in levels] == [(320, 240), (266, 200), (222, 166)]
    assert len(cands) == math.ceil(0.01 * 855)
    assert 1 <= len(kept) <= len(cands)
    for a in range(len(kept)):
        for b in range(a + 1, len(kept)):
            assert not O.iou_exceeds_half(kept[a]["box"], kept[b]["box"])
