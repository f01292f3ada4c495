"""The single-family pipelines (HOG-SVM, LBP-SVM): pd_params.features set to
one family makes every kernel skip the other, which is the full detector with
that family's weights at zero (the linear model then ignores those features).
So the full-feature FP64 oracle with the masked weights is the reference, at
the tolerances of the full pipeline (window lists and NMS exact, scores within
1e-4)."""
import math

import numpy as np
import pytest

import pd_synth
from oracle import pd_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_01642_amd as pd  # noqa: E402

DEV = "cuda:0"
HOG_DIM = 15 * 7 * 36


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def masked(wts, feat):
    w = np.array(wts, np.float32, copy=True)
    if feat == pd.FEAT_HOG:
        w[:, HOG_DIM:] = 0.0
    else:
        w[:, :HOG_DIM] = 0.0
    return w


def run_detect(frames, wts, bias, thr, prm):
    det = pd.Detector([to_dev(f) for f in frames], to_dev(wts), to_dev(bias), prm, cap=1024)
    det.run(to_dev(np.asarray(thr, np.float64)))
    torch.cuda.synchronize()
    return det.results()


def check_frame(boxes, counts, levels, cands, kept):
    assert counts["candidates"] == len(cands)
    assert counts["overflow"] == 0
    assert [(int(b["level"]), int(b["i"]), int(b["j"]), int(b["model"])) for b in boxes] == \
        [(c["level"], c["i"], c["j"], c["model"]) for c in kept]
    for b, c in zip(boxes, kept):
        assert (b["x0"], b["y0"], b["x1"], b["y1"]) == c["box"]
        assert abs(b["score"] - c["score"]) <= 1e-4 * max(abs(c["score"]), 1.0)


@pytest.mark.parametrize("feat", [pd.FEAT_HOG, pd.FEAT_LBP], ids=["hog", "lbp"])
@pytest.mark.parametrize("cfg", ["small", "road"])
def test_subset_detect_matches_oracle(feat, cfg):
    if cfg == "small":
        w, h, scale, maxl = 320, 240, (6, 5), 3
    else:
        w, h, scale, maxl = 1242, 375, (11, 10), 0
    print(f"subset {feat} {cfg}", flush=True)
    img = pd_synth.frame(w, h, 1200 + feat)
    wts = masked(pd_synth.svm_weights(1), feat)
    bias = pd_synth.svm_bias(1)
    levels, thr, cands, kept = O.detect(img, wts, bias, scale_num=scale[0], scale_den=scale[1], max_levels=maxl)
    assert len(cands) == math.ceil(0.01 * sum(lv["scores"].size for lv in levels))
    boxes, counts = run_detect([img], wts, bias, [thr], pd.params(scale=scale, max_levels=maxl, features=feat))
    check_frame(boxes[0], counts[0], levels, cands, kept)


@pytest.mark.parametrize("feat", [pd.FEAT_HOG, pd.FEAT_LBP], ids=["hog", "lbp"])
def test_subset_batch_multi_model(feat):
    """Two frames of different sizes in one call, three models with biases;
    the unmasked weights give the same result (the skipped family's weights
    are never read)."""
    sizes = [(333, 257), (640, 480)]
    frames = [pd_synth.frame(w, h, 1300 + w) for w, h in sizes]
    raw = pd_synth.svm_weights(3)
    wts = masked(raw, feat)
    bias = np.array([0.2, -0.1, 0.0], np.float32)
    refs = [O.detect(f, wts, bias) for f in frames]
    thr = [r[1] for r in refs]
    prm = pd.params(features=feat)
    boxes, counts = run_detect(frames, wts, bias, thr, prm)
    boxes_raw, _ = run_detect(frames, raw, bias, thr, prm)
    for f, (levels, _, cands, kept) in enumerate(refs):
        check_frame(boxes[f], counts[f], levels, cands, kept)
        assert boxes[f].tobytes() == boxes_raw[f].tobytes()
