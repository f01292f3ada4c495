"""FP32 window scores of pd_detect (the matrix-core scoring kernel), every window.

* With every window a candidate, each window's score (the max over models)
  and its model equal the FP64 oracle's within the scoring tolerance, for a
  road frame with two models and biases (one frame: the kernel splits each
  row of tiles into runs, each recomputing the tile to its left).
* Each window's FP32 sum runs in one order whatever the band height, the
  grid, the run split or the batch: the scores of a 17-frame mixed batch are
  the same bits for every band height and grid cap, and equal the bits of
  the frames scored one at a time.
"""
import numpy as np
import pytest

import pd_synth
from oracle import pd_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_01642_amd as pd  # noqa: E402

DEV = "cuda:0"
CLIP32, EPS32 = float(np.float32(0.2)), float(np.float32(1e-3))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def all_windows(frames, wts, bias, prm):
    """Per frame: (keys [n][4] = level, i, j, model; FP32 scores [n]), sorted by key."""
    det = pd.Detector([to_dev(f) for f in frames], to_dev(wts), to_dev(bias), prm, cap=1)
    det.run(to_dev(np.full(len(frames), -1e30)))
    torch.cuda.synchronize()
    out = []
    for f in range(len(frames)):
        cs, ck, _ = det.candidates(f)
        keys = np.asarray(ck, np.int64)[:, :4]
        order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
        out.append((keys[order], np.asarray(cs, np.float32)[order]))
    det.release()
    return out


def test_every_window_matches_oracle():
    img = pd_synth.frame(1242, 375, 7100)
    wts = pd_synth.svm_weights(2)
    bias = np.array([0.25, -0.4], np.float32)
    levels = O.frame_scores(img, wts, bias, clip=CLIP32, eps=EPS32)
    (keys, got), = all_windows([img], wts, bias, pd.params())
    ref_s, ref_m = [], []
    for k, lv in enumerate(levels):
        s = lv["scores"]  # [m][Y][X]
        ref_s.append(s.max(axis=0).ravel())
        ref_m.append(s.argmax(axis=0).ravel())
        assert np.count_nonzero(keys[:, 0] == k) == s[0].size
    ref_s, ref_m = np.concatenate(ref_s), np.concatenate(ref_m)
    assert len(got) == len(ref_s) == 18451
    sigma = ref_s.std()
    err = np.abs(got.astype(np.float64) - ref_s)
    tol = 1e-4 * np.maximum(np.abs(ref_s), sigma)
    print(f"\n[score32] 1242x375, 2 models: max err {err.max():.3g} ({err.max() / sigma:.2g} sigma)", flush=True)
    assert np.all(err <= tol)
    # the model with the larger score, where the two are not within rounding of each other
    s2 = np.concatenate([lv["scores"].reshape(2, -1) for lv in levels], axis=1)
    clear = np.abs(s2[0] - s2[1]) > 1e-3 * np.maximum(np.abs(s2).max(axis=0), sigma)
    assert np.array_equal(keys[clear, 3], ref_m[clear])


def test_same_bits_for_any_band_grid_run_and_batch():
    sizes = [(1242, 375), (640, 480), (320, 240), (333, 257), (64, 128), (130, 135)] * 3
    frames = pd_synth.frame_batch(sizes[:17], 7200)
    wts = pd_synth.svm_weights(1)
    bias = np.array([0.1], np.float32)
    ref = all_windows(frames, wts, bias, pd.params())
    for kw in (dict(tune_score_rows=4), dict(tune_score_rows=16), dict(tune_grid=8), dict(tune_grid=24),
               dict(tune_score_rows=4, tune_grid=16)):
        print(f"\n[score32] 17 frames {kw}", flush=True)
        got = all_windows(frames, wts, bias, pd.params(**kw))
        for f in range(len(frames)):
            assert np.array_equal(got[f][0], ref[f][0]), f
            assert got[f][1].tobytes() == ref[f][1].tobytes(), (kw, f)
    for f in (0, 1, 3):
        (k1, s1), = all_windows([frames[f]], wts, bias, pd.params())
        assert np.array_equal(k1, ref[f][0]) and s1.tobytes() == ref[f][1].tobytes(), f
