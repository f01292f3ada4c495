"""BF16 MFMA scoring with FP64 rescoring of near-threshold windows, through
the C ABI, against the FP64 oracle.

Checks:
* BF16 HOG planes are the FP32 ones rounded to nearest even (bitwise);
* the MFMA scoring kernel, fed BF16-rounded oracle features, equals the
  exact sum of those BF16 features times the hi+lo BF16 weight split up to
  FP32 accumulation (isolates the kernel's operand layout);
* on the road frame with 8 models, every decision (window above the
  threshold) equals the oracle's; rescored windows carry the oracle's FP64
  score; the BF16 error of every window is inside a rigorous bound.
"""
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


def bf16_round(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def test_bf16_hog_is_rne_of_fp32():
    img = to_dev(pd_synth.frame(640, 480, 12))
    f32, c1 = pd.features(img)
    b16, c2 = pd.features(img, bf16=True)
    assert b16.dtype == torch.bfloat16
    assert torch.equal(f32.to(torch.bfloat16).view(torch.int16), b16.view(torch.int16))
    assert torch.equal(c1, c2)


@pytest.mark.parametrize("w,h,m", [(64, 128, 1), (333, 257, 8), (1242, 375, 3)])
def test_mfma_scoring_exact_operands(w, h, m):
    img = pd_synth.frame(w, h, 40 + w)
    hog = O.hog_features(img)
    cells = O.lbp_cell_histograms(img).astype(np.uint8)
    hog16 = bf16_round(hog)                                  # the BF16 features the kernel reads
    wts = pd_synth.svm_weights(m)
    bias = np.linspace(-1.0, 1.0, m).astype(np.float32)
    hi = bf16_round(wts)
    lo = bf16_round(wts.astype(np.float64) - hi)
    lo[:, :O.HOG_DIM] = 0.0          # HOG weights carry their BF16 part only
    packed = pd.pack_models(to_dev(wts))
    got = pd.score_windows_bf16(to_dev(hog16.astype(np.float32).transpose(2, 0, 1)).to(torch.bfloat16),
                                to_dev(cells.transpose(2, 0, 1)), packed, to_dev(bias), m).cpu().numpy()
    exp = O.window_scores(hog16, cells, hi + lo, bias.astype(np.float64))
    absx = O.window_scores(np.abs(hog16), cells, np.abs(hi) + np.abs(lo), np.zeros(m))
    assert got.shape == exp.shape
    err = np.abs(got - exp)
    # FP32 accumulation of ~2 x 11520 exact products: a loose a-priori bound
    assert np.all(err <= 2 * 11520 * 2.0 ** -24 * absx + 1e-6), err.max()
    # and in practice far below it
    assert err.max() <= 1e-5 * max(1.0, absx.max()), (err.max(), absx.max())


# The library takes L2-Hys clip and eps as FP32 parameters (pd_params), so its
# FP64 rescore works with their FP32 values widened exactly; the oracle gets
# the same values wherever FP64 scores are compared at 1e-9.
CLIP32, EPS32 = float(np.float32(0.2)), float(np.float32(1e-3))


def _oracle_frame(img, m, scale=(11, 10), maxl=0):
    wts, bias = pd_synth.svm_weights(m), np.zeros(m, np.float32)
    levels = O.frame_scores(img, wts, bias, scale[0], scale[1], maxl, clip=CLIP32, eps=EPS32)
    thr = O.frame_threshold(levels)
    return wts, bias, levels, thr


@pytest.mark.parametrize("cfg", ["small8", "road8", "road1"])
def test_detect_bf16_decisions_equal_oracle(cfg):
    if cfg == "small8":
        img, scale, maxl = pd_synth.frame(320, 240, 1000), (6, 5), 3
    else:
        img, scale, maxl = pd_synth.frame(1242, 375, 1000), (11, 10), 0
    m = 1 if cfg.endswith("1") else 8
    wts, bias, levels, thr = _oracle_frame(img, m, scale, maxl)
    h0, w0 = img.shape
    prm = pd.params(scale=scale, max_levels=maxl, precision=pd.PREC_BF16, margin=0.05)
    det = pd.Detector([to_dev(img)], to_dev(wts), to_dev(bias), prm, cap=1024)
    det.run(to_dev(np.array([thr])))
    torch.cuda.synchronize()
    boxes, counts = det.results()
    cs, ck, c64 = det.candidates(0)

    oracle_c = O.candidates(levels, w0, h0, thr)
    exp = {(c["level"], c["i"], c["j"]): c for c in oracle_c}
    got = {(int(k[0]), int(k[1]), int(k[2])): (float(s), int(k[3]), float(s64)) for s, k, s64 in zip(cs, ck, c64)}
    assert counts[0]["overflow"] == 0
    assert set(got) == set(exp), (len(set(got) - set(exp)), len(set(exp) - set(got)))
    assert counts[0]["candidates"] == len(exp)

    # errors of every window (all levels, all models) against the oracle
    sig = np.concatenate([lv["scores"].max(axis=0).ravel() for lv in levels]).std()
    pyr = pd.build_pyramid(to_dev(img), prm)[2]
    packed = pd.pack_models(to_dev(wts))
    worst_ratio, errs = 0.0, []
    for k, (v, lv) in enumerate(zip(pyr, levels)):
        b16, cel = pd.features(v.contiguous(), prm, bf16=True)
        s = pd.score_windows_bf16(b16, cel, packed, to_dev(bias), m).cpu().numpy().astype(np.float64)
        ref = lv["scores"]
        absx = O.window_scores(lv["hog"], lv["cells"], np.abs(wts.astype(np.float64)), np.zeros(m))
        hog_only = O.window_scores(lv["hog"], np.zeros_like(lv["cells"]), np.abs(wts.astype(np.float64)),
                                   np.zeros(m))
        # HOG features rounded to BF16 (2^-9 relative) + their FP32 computation (1e-5),
        # HOG weights rounded to BF16 (2^-9), LBP weights as hi + lo (2^-17), FP32
        # accumulation of ~2 x 11520 products
        bound = (2.0 ** -8 + 1e-5) * hog_only + 2.0 ** -17 * absx + 2 * 11520 * 2.0 ** -24 * absx
        err = np.abs(s - ref)
        assert np.all(err <= bound), (k, err.max())
        worst_ratio = max(worst_ratio, float((err / bound).max()))
        errs.append(err.ravel())
    errs = np.concatenate(errs)
    # decisions and FP64 rescores
    n_res = 0
    for key, (s, model, s64) in got.items():
        ref = exp[key]["score"]
        if not math.isnan(s64):
            n_res += 1
            assert abs(s64 - ref) <= 1e-9 * max(1.0, abs(ref)), (key, s64, ref)
            assert model == exp[key]["model"]
        else:
            assert abs(s - ref) < 0.05
    print(f"\n[bf16 report] {cfg}: windows {errs.size // m} x {m} models, candidates {len(exp)}, "
          f"rescored {counts[0]['rescored']} (candidates among them {n_res}); |s_bf16 - s_oracle|: "
          f"max {errs.max():.3g}, mean {errs.mean():.3g}, max/sigma {errs.max() / sig:.3g}; "
          f"worst err/bound {worst_ratio:.3g}; kept {counts[0]['kept']}")
    # NMS of the rescored candidate list: a valid greedy result
    kept = [(int(b["level"]), int(b["i"]), int(b["j"])) for b in boxes[0]]
    assert set(kept) <= set(got)
    for a in range(len(boxes[0])):
        for b in range(a + 1, len(boxes[0])):
            ba = tuple(int(boxes[0][a][q]) for q in ("x0", "y0", "x1", "y1"))
            bb = tuple(int(boxes[0][b][q]) for q in ("x0", "y0", "x1", "y1"))
            assert not O.iou_exceeds_half(ba, bb)


def test_detect_bf16_batch_deterministic():
    frames = pd_synth.frame_batch([(1242, 375), (640, 480), (1242, 375)], 3000)
    wts = pd_synth.svm_weights(8)
    bias = np.zeros(8, np.float32)
    prm = pd.params(precision=pd.PREC_BF16)
    # thresholds near the 95th percentile of the 8-model max score: every
    # candidate list within what NMS takes whole
    thr = to_dev(np.array([6.3, 6.3, 6.3]))
    dets = []
    for _ in range(2):
        det = pd.Detector([to_dev(f) for f in frames], to_dev(wts), to_dev(bias), prm, cap=1024)
        det.run(thr)
        torch.cuda.synchronize()
        dets.append(det.results())
    for f in range(3):
        assert dets[0][1][f]["overflow"] == 0 and dets[0][1][f]["candidates"] > 0
        assert dets[0][0][f].tobytes() == dets[1][0][f].tobytes()
    single = pd.Detector([to_dev(frames[1])], to_dev(wts), to_dev(bias), prm, cap=1024)
    single.run(thr[:1])
    torch.cuda.synchronize()
    b1, c1 = single.results()
    b = dets[0][0][1].copy()
    b["frame"] = 0
    assert b.tobytes() == b1[0].tobytes()


@pytest.mark.parametrize("w,h,m", [(166, 203, 8), (201, 150, 1)])
def test_rescore_every_window(w, h, m):
    """A margin that makes every window near the threshold: all windows of a
    small frame (border windows, whose pixels are clamped, and inner ones,
    read as aligned words) go through the FP64 rescore; every candidate
    carries the oracle's FP64 score and model, and the candidate set is the
    oracle's exactly (the threshold lies midway between two oracle scores)."""
    img = pd_synth.frame(w, h, 4321 + w)
    wts, bias = pd_synth.svm_weights(m), np.zeros(m, np.float32)
    levels = O.frame_scores(img, wts, bias.astype(np.float64), clip=CLIP32, eps=EPS32)
    allmax = np.sort(np.concatenate([O.max_over_models(lv["scores"])[0].ravel() for lv in levels]))
    n_win = allmax.size
    assert n_win > 0
    k = n_win // 3
    thr = 0.5 * (allmax[n_win - k - 1] + allmax[n_win - k])
    prm = pd.params(precision=pd.PREC_BF16, margin=1.0e6)
    det = pd.Detector([to_dev(img)], to_dev(wts), to_dev(bias), prm, cap=1024)
    det.run(to_dev(np.array([thr])))
    torch.cuda.synchronize()
    _, counts = det.results()
    assert counts[0]["rescored"] == n_win and counts[0]["overflow"] == 0
    cs, ck, c64 = det.candidates(0)
    exp = {(c["level"], c["i"], c["j"]): c for c in O.candidates(levels, w, h, thr)}
    got = {(int(q[0]), int(q[1]), int(q[2])): (float(s), int(q[3])) for q, s in zip(ck, c64)}
    assert set(got) == set(exp)
    for key, (s64, model) in got.items():
        ref = exp[key]["score"]
        assert abs(s64 - ref) <= 1e-9 * max(1.0, abs(ref)), (key, s64, ref)
        assert model == exp[key]["model"]
    print(f"\n[rescore all] {w}x{h} m {m}: windows {n_win}, candidates {len(exp)}", flush=True)
