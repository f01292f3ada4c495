"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: integer results (pyramid, LBP codes and histograms, window lists,
NMS decisions) are bit-exact; HOG features within 1e-4 |x_ref| + 1e-6; window
scores within 1e-4 max(|s_ref|, sigma_s), sigma_s the oracle score std of the
level (FP32 products and sums over 11332 terms vs FP64)."""
import math

import numpy as np
import pytest

import pd_synth
from oracle import pd_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_01642_amd as pd  # noqa: E402

DEV = "cuda:0"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def note(msg):
    print(msg, flush=True)


def hog_close(got, ref):
    ref = np.asarray(ref, np.float64)
    err = np.abs(got.astype(np.float64) - ref)
    bad = err > 1e-4 * np.abs(ref) + 1e-6
    assert not bad.any(), f"{bad.sum()} HOG values off, max err {err.max():.3g}"


def scores_close(got, ref):
    ref = np.asarray(ref, np.float64)
    sigma = ref.std() if ref.size > 1 else 1.0
    err = np.abs(got.astype(np.float64) - ref)
    tol = 1e-4 * np.maximum(np.abs(ref), sigma)
    assert np.all(err <= tol), f"max score err {err.max():.3g} (sigma {sigma:.3g})"
    return err.max() / max(sigma, 1e-30)


SIZES = [(320, 240), (333, 257), (17, 9), (64, 128), (130, 135), (1242, 375)]


# ---------------------------------------------------------------- pyramid --

@pytest.mark.parametrize("w,h,scale,maxl", [(320, 240, (6, 5), 3), (1242, 375, (11, 10), 0),
                                            (1001, 299, (12, 10), 0), (64, 128, (11, 10), 0)])
def test_pyramid_bit_exact(w, h, scale, maxl):
    note(f"pyramid {w}x{h} scale {scale}")
    img = pd_synth.frame(w, h, 1000 + w)
    _, levels, views = pd.build_pyramid(to_dev(img), pd.params(scale=scale, max_levels=maxl))
    torch.cuda.synchronize()
    exp = O.pyramid(img, scale[0], scale[1], maxl)
    assert len(views) == len(exp)
    for k, (v, e) in enumerate(zip(views, exp)):
        assert np.array_equal(v.cpu().numpy(), e), f"level {k}"


def test_pyramid_pitched_input():
    img = pd_synth.frame(400, 300, 5)
    padded = np.zeros((300, 432), np.uint8)
    padded[:, :400] = img
    t = to_dev(padded)[:, :400]
    _, _, views = pd.build_pyramid(t)
    torch.cuda.synchronize()
    for v, e in zip(views, O.pyramid(img)):
        assert np.array_equal(v.cpu().numpy(), e)


# -------------------------------------------------------------------- LBP --

@pytest.mark.parametrize("w,h", [(1, 1), (7, 9)] + SIZES)
def test_lbp_codes_bit_exact(w, h):
    note(f"lbp codes {w}x{h}")
    img = pd_synth.frame(w, h, 77 + w)
    got = pd.lbp_codes(to_dev(img)).cpu().numpy()
    assert np.array_equal(got, O.lbp_codes(img))


@pytest.mark.parametrize("w,h", SIZES)
def test_lbp_histograms_bit_exact(w, h):
    note(f"lbp hist {w}x{h}")
    img = pd_synth.frame(w, h, 11 + h)
    got = pd.lbp(to_dev(img)).cpu().numpy()
    ref = O.lbp_cell_histograms(img)
    assert got.shape == (59, h // 8, w // 8)
    assert np.array_equal(got.transpose(1, 2, 0).astype(np.int64), ref)
    assert np.all(got.sum(axis=0, dtype=np.int64) == 64)


def test_lbp_constant_and_uniform_noise():
    img = np.full((48, 80), 200, np.uint8)
    got = pd.lbp(to_dev(img)).cpu().numpy()
    assert np.all(got[57] == 64) and got.sum() == 64 * 6 * 10
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, size=(131, 259), dtype=np.uint8)
    assert np.array_equal(pd.lbp(to_dev(img)).cpu().numpy().transpose(1, 2, 0), O.lbp_cell_histograms(img))


# -------------------------------------------------------------------- HOG --

@pytest.mark.parametrize("w,h", [s for s in SIZES if s[0] >= 16 and s[1] >= 16])
def test_hog_matches_oracle(w, h):
    note(f"hog {w}x{h}")
    img = pd_synth.frame(w, h, 31 + w)
    got = pd.hog(to_dev(img)).cpu().numpy().transpose(1, 2, 0)
    hog_close(got, O.hog_features(img))


def test_hog_random_noise_and_pitch():
    rng = np.random.default_rng(2)
    img = rng.integers(0, 256, size=(140, 260), dtype=np.uint8)
    padded = np.zeros((140, 272), np.uint8)
    padded[:, :260] = img
    got = pd.hog(to_dev(padded)[:, :260]).cpu().numpy().transpose(1, 2, 0)
    hog_close(got, O.hog_features(img))


def test_hog_closed_forms():
    img = np.tile(np.arange(160, dtype=np.uint8), (64, 1))
    f = pd.hog(to_dev(img)).cpu().numpy().transpose(1, 2, 0)[1:-1, 1:-1]
    nzi = [0, 8, 9, 17, 18, 26, 27, 35]
    assert np.allclose(f[..., nzi], 0.2 / math.sqrt(0.320001), rtol=1e-5, atol=0)
    mask = np.ones(36, bool)
    mask[nzi] = False
    assert np.abs(f[..., mask]).max() < 1e-6
    img = np.tile(np.arange(96, dtype=np.uint8)[:, None], (1, 48))
    f = pd.hog(to_dev(img)).cpu().numpy().transpose(1, 2, 0)[1:-1, 1:-1]
    assert np.allclose(f[..., [4, 13, 22, 31]], 0.49999844, rtol=1e-5, atol=0)
    assert np.all(pd.hog(to_dev(np.full((40, 48), 9, np.uint8))).cpu().numpy() == 0)


def test_feature_subsets_agree():
    img = to_dev(pd_synth.frame(300, 200, 3))
    b_all, c_all = pd.features(img)
    b_h, _ = pd.features(img, hog=True, lbp=False)
    _, c_l = pd.features(img, hog=False, lbp=True)
    assert torch.equal(b_all, b_h) and torch.equal(c_all, c_l)


def test_features_deterministic():
    img = to_dev(pd_synth.frame(1242, 375, 9))
    a = pd.features(img)
    b = pd.features(img)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


# ---------------------------------------------------------------- scoring --

@pytest.mark.parametrize("w,h,m", [(64, 128, 1), (333, 257, 3), (1242, 375, 1)])
def test_scores_on_oracle_features(w, h, m):
    """Scoring alone: both sides score the same FP32 HOG / uint8 LBP features."""
    note(f"scores {w}x{h} m={m}")
    img = pd_synth.frame(w, h, 5 + w)
    hog = O.hog_features(img).astype(np.float32)
    cells = O.lbp_cell_histograms(img).astype(np.uint8)
    wts = pd_synth.svm_weights(m)
    bias = np.linspace(-0.5, 0.5, m).astype(np.float32)
    got = pd.score_windows(to_dev(hog.transpose(2, 0, 1)), to_dev(cells.transpose(2, 0, 1)),
                           to_dev(wts), to_dev(bias)).cpu().numpy()
    ref = O.window_scores(hog.astype(np.float64), cells, wts, bias)
    assert got.shape == ref.shape
    for k in range(m):
        scores_close(got[k], ref[k])


def test_scores_indicator_weights_gather():
    img = pd_synth.frame(200, 180, 8)
    hog = O.hog_features(img).astype(np.float32)
    cells = O.lbp_cell_histograms(img).astype(np.uint8)
    w = np.zeros((2, 11332), np.float32)
    w[0, (3 * 7 + 5) * 36 + 17] = 1.0
    w[1, 3780 + (11 * 8 + 2) * 59 + 58] = 1.0
    got = pd.score_windows(to_dev(hog.transpose(2, 0, 1)), to_dev(cells.transpose(2, 0, 1)), to_dev(w),
                           to_dev(np.zeros(2, np.float32))).cpu().numpy()
    ny, nx = got.shape[1:]
    assert np.array_equal(got[0], hog[3:3 + ny, 5:5 + nx, 17])
    assert np.array_equal(got[1], cells[11:11 + ny, 2:2 + nx, 58].astype(np.float32))


# ------------------------------------------------------------ whole path --

def oracle_frame(img, wts, bias, scale=(11, 10), maxl=0):
    return O.detect(img, wts, bias, scale_num=scale[0], scale_den=scale[1], max_levels=maxl)


def run_detect(frames, wts, bias, thr, prm, cap=1024):
    det = pd.Detector([to_dev(f) for f in frames], to_dev(wts), to_dev(bias), prm, cap=cap)
    det.run(to_dev(np.asarray(thr, np.float64)))
    torch.cuda.synchronize()
    return det.results()


def run_detect_views(views, wts, bias, thr, prm, cap=1024):
    det = pd.Detector(views, to_dev(wts), to_dev(bias), prm, cap=cap)
    det.run(to_dev(np.asarray(thr, np.float64)))
    torch.cuda.synchronize()
    return det.results()


def kept_keys(boxes):
    return [(int(b["level"]), int(b["i"]), int(b["j"])) for b in boxes]


@pytest.mark.parametrize("cfg", ["small", "road"])
def test_detect_matches_oracle(cfg):
    if cfg == "small":
        w, h, scale, maxl = 320, 240, (6, 5), 3
    else:
        w, h, scale, maxl = 1242, 375, (11, 10), 0
    note(f"detect {cfg}")
    img = pd_synth.frame(w, h, 1000)
    wts, bias = pd_synth.svm_weights(1), pd_synth.svm_bias(1)
    levels, thr, cands, kept = oracle_frame(img, wts, bias, scale, maxl)
    prm = pd.params(scale=scale, max_levels=maxl)
    boxes, counts = run_detect([img], wts, bias, [thr], prm)
    assert counts[0]["candidates"] == len(cands) == math.ceil(0.01 * sum(lv["scores"].size for lv in levels))
    assert counts[0]["overflow"] == 0
    assert kept_keys(boxes[0]) == [(c["level"], c["i"], c["j"]) for c in kept]
    for b, c in zip(boxes[0], kept):
        assert (b["x0"], b["y0"], b["x1"], b["y1"]) == c["box"]
        assert abs(b["score"] - c["score"]) <= 1e-4 * max(abs(c["score"]), 1.0)
        assert np.isnan(b["score64"])
    # per-level window lists, from the GPU's own features and scores
    pyr, _, views = pd.build_pyramid(to_dev(img), prm)
    for k, (v, lv) in enumerate(zip(views, levels)):
        blocks, cells = pd.features(v.contiguous(), prm)
        s = pd.score_windows(blocks, cells, to_dev(wts), to_dev(bias)).cpu().numpy()[0]
        ref = lv["scores"][0]
        scores_close(s, ref)
        assert np.array_equal(np.argwhere(s.astype(np.float64) > thr), np.argwhere(ref > thr)), f"level {k}"


def test_detect_multi_model_and_bias():
    img = pd_synth.frame(400, 300, 1001)
    wts = pd_synth.svm_weights(3)
    bias = np.array([0.3, -0.2, 0.1], np.float32)
    levels, thr, cands, kept = oracle_frame(img, wts, bias)
    boxes, counts = run_detect([img], wts, bias, [thr], pd.params())
    assert counts[0]["candidates"] == len(cands)
    assert [(int(b["level"]), int(b["i"]), int(b["j"]), int(b["model"])) for b in boxes[0]] == \
        [(c["level"], c["i"], c["j"], c["model"]) for c in kept]


def test_detect_batched_mixed_sizes_equal_single():
    sizes = [(640, 480), (1242, 375), (64, 128), (50, 50), (333, 257)]
    frames = pd_synth.frame_batch(sizes, 2000)
    wts, bias = pd_synth.svm_weights(1), pd_synth.svm_bias(1)
    thr = [0.5, 1.0, -100.0, 0.0, 2.0]
    batch, counts = run_detect(frames, wts, bias, thr, pd.params())
    again, counts2 = run_detect(frames, wts, bias, thr, pd.params())
    for f in range(len(frames)):
        single, c1 = run_detect([frames[f]], wts, bias, [thr[f]], pd.params())
        assert counts[f]["candidates"] == c1[0]["candidates"]
        b = batch[f].copy()
        b["frame"] = 0
        assert b.tobytes() == single[0].tobytes(), f"frame {f}"
        assert batch[f].tobytes() == again[f].tobytes()
    assert counts[3]["candidates"] == 0 and counts[3]["kept"] == 0   # smaller than a window
    assert counts[2]["candidates"] == 1 and counts[2]["kept"] == 1   # exactly one window


def test_nms_matches_oracle_random():
    rng = np.random.default_rng(4)
    wh = [(1242, 375), (1129, 340), (1026, 309)]
    for trial in range(6):
        n = [0, 1, 63, 64, 65, 700][trial]
        cands = []
        for q in range(n):
            k = int(rng.integers(0, 3))
            ny, nx = O.window_grid(*wh[k])
            i, j = int(rng.integers(0, ny)), int(rng.integers(0, nx))
            s = float(np.float32(rng.normal() if q % 7 else 1.25))  # some exact ties
            cands.append({"score": s, "level": k, "i": i, "j": j, "model": q % 2,
                          "box": O.window_box_q8(1242, 375, wh[k][0], wh[k][1], i, j)})
        # drop duplicate windows (a window is one candidate)
        seen, uniq = set(), []
        for c in cands:
            if (c["level"], c["i"], c["j"]) not in seen:
                seen.add((c["level"], c["i"], c["j"]))
                uniq.append(c)
        n = len(uniq)
        cs = to_dev(np.array([c["score"] for c in uniq], np.float32).reshape(n))
        ck = to_dev(np.array([[c["level"], c["i"], c["j"], c["model"]] for c in uniq], np.int32).reshape(n, 4))
        boxes, counts = pd.nms(cs, ck, wh, cap=1024)
        got, cnt = pd.decode_boxes(boxes, counts)
        exp = O.nms(uniq)
        assert cnt["candidates"] == n and cnt["kept"] == len(exp)
        assert [(int(b["level"]), int(b["i"]), int(b["j"])) for b in got] == [(c["level"], c["i"], c["j"]) for c in exp]
        assert [tuple(int(b[k]) for k in ("x0", "y0", "x1", "y1")) for b in got] == [c["box"] for c in exp]


def test_nms_full_list_with_ties():
    """A list of PD_MAX_CANDIDATES distinct windows over three levels, scores
    from a small set (many exact ties, +0 and -0 among them, which tie):
    the kept list, in order, equals the oracle's greedy NMS."""
    rng = np.random.default_rng(44)
    wh = [(1242, 375), (1129, 340), (1026, 309)]
    allw = [(k, i, j) for k, (w, h) in enumerate(wh) for i in range(O.window_grid(w, h)[0])
            for j in range(O.window_grid(w, h)[1])]
    pick = rng.choice(len(allw), size=pd.MAX_CANDIDATES, replace=False)
    values = np.array([-0.0, 0.0, 1.25, -2.5, 3.0, 0.5], np.float32)
    cands = []
    for q, p in enumerate(pick):
        k, i, j = allw[int(p)]
        s = float(values[q % len(values)]) if q % 3 else float(np.float32(rng.normal()))
        cands.append({"score": s, "level": k, "i": i, "j": j, "model": 0,
                      "box": O.window_box_q8(1242, 375, wh[k][0], wh[k][1], i, j)})
    n = len(cands)
    cs = to_dev(np.array([c["score"] for c in cands], np.float32))
    ck = to_dev(np.array([[c["level"], c["i"], c["j"], 0] for c in cands], np.int32))
    boxes, counts = pd.nms(cs, ck, wh, cap=n)
    got, cnt = pd.decode_boxes(boxes, counts)
    exp = O.nms(cands)
    assert cnt["candidates"] == n and cnt["overflow"] == 0 and cnt["kept"] == len(exp)
    assert [(int(b["level"]), int(b["i"]), int(b["j"])) for b in got] == [(c["level"], c["i"], c["j"]) for c in exp]


def test_nms_cap_reports_overflow():
    wh = [(1242, 375)]
    n = 40
    cs = to_dev(np.arange(n, dtype=np.float32))
    ck = to_dev(np.array([[0, 0, 8 * q, 0] for q in range(n)], np.int32).reshape(n, 4))  # disjoint boxes
    boxes, counts = pd.nms(cs, ck, wh, cap=10)
    got, cnt = pd.decode_boxes(boxes, counts)
    assert cnt["kept"] == 10 and cnt["overflow"] == 1
    assert [int(b["j"]) for b in got] == [8 * q for q in range(n - 1, n - 11, -1)]


@pytest.mark.parametrize("prec", [pd.PREC_F32, pd.PREC_BF16])
def test_detect_pitched_misaligned_frames_equal_contiguous(prec):
    """Frames given as views into wider buffers, starting 1-3 bytes past an
    aligned address with pitches that are not multiples of 4: the same boxes
    and counts, bytewise, as the contiguous frames."""
    sizes = [(1242, 375), (640, 480), (333, 257)]
    frames = pd_synth.frame_batch(sizes, 2100)
    wts, bias = pd_synth.svm_weights(1), pd_synth.svm_bias(1)
    thr = [3.0, 3.0, 3.0]  # every frame's candidates within what NMS takes whole
    prm = pd.params(precision=prec, margin=0.05) if prec == pd.PREC_BF16 else pd.params()
    views, bufs = [], []
    for k, img in enumerate(frames):
        h, w = img.shape
        off, pitch = 1 + k, w + 7 + 2 * k
        buf = torch.zeros(h * pitch + 64, dtype=torch.uint8, device=DEV)
        v = buf[off:off + h * pitch].view(h, pitch)[:, :w]
        v.copy_(to_dev(img))
        assert v.data_ptr() % 4 == off % 4 and v.stride(0) == pitch
        views.append(v)
        bufs.append(buf)
    got_b, got_c = run_detect_views(views, wts, bias, thr, prm)
    exp_b, exp_c = run_detect(frames, wts, bias, thr, prm)
    assert np.all(exp_c["overflow"] == 0) and np.all(exp_c["kept"] > 0)
    assert got_c.tobytes() == exp_c.tobytes()
    for f in range(len(frames)):
        assert got_b[f].tobytes() == exp_b[f].tobytes(), f"frame {f}"
