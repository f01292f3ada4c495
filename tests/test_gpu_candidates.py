"""Candidate lists without drops, and the overflow contract.

* Every window within the margin of the threshold is rescored in FP64, however
  many there are: a 1242x375 BF16 frame with a margin that makes all 18,451
  windows near (1 and 8 models) gives the oracle's candidate set with every
  candidate's FP64 score within 1e-9.
* A frame with more than PD_MAX_CANDIDATES candidates keeps all of them in its
  list (the true count), and NMS runs on the PD_MAX_CANDIDATES highest-scoring
  ones in the NMS order (score descending, then level, i, j): the kept boxes
  equal the oracle's greedy NMS of that selection of the device's candidates,
  and two runs give the same bytes (FP32 and BF16 with rescoring).
* A graph captured before an autotuning run (which captures and launches
  graphs of other tile shapes on the same workspace) still replays to the
  eager result: it owns its tables.
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
CLIP32, EPS32 = float(np.float32(0.2)), float(np.float32(1e-3))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def run(frames, wts, bias, thr, prm, cap=1024):
    det = pd.Detector([to_dev(f) for f in frames], to_dev(wts), to_dev(bias), prm, cap=cap)
    det.run(to_dev(np.asarray(thr, np.float64)))
    torch.cuda.synchronize()
    return det, det.results()


@pytest.mark.parametrize("m", [1, 8])
def test_rescore_every_window_of_a_road_frame(m):
    img = pd_synth.frame(1242, 375, 4500 + m)
    wts, bias = pd_synth.svm_weights(m), np.zeros(m, np.float32)
    levels = O.frame_scores(img, wts, bias, clip=CLIP32, eps=EPS32)
    n_win = sum(lv["scores"][0].size for lv in levels)
    assert n_win == 18451
    thr = O.frame_threshold(levels)
    print(f"\n[rescore all] 1242x375, {m} models, {n_win} windows", flush=True)
    det, (boxes, counts) = run([img], wts, bias, [thr], pd.params(precision=pd.PREC_BF16, margin=1.0e6))
    c = counts[0]
    exp = {(e["level"], e["i"], e["j"]): e for e in O.candidates(levels, 1242, 375, thr)}
    assert len(exp) == math.ceil(0.01 * n_win)
    assert c["rescored"] == n_win and c["overflow"] == 0 and c["candidates"] == len(exp)
    cs, ck, c64 = det.candidates(0)
    got = {(int(k[0]), int(k[1]), int(k[2])): (float(s), int(k[3])) for k, s in zip(ck, c64)}
    assert set(got) == set(exp)
    worst = 0.0
    for key, (s64, model) in got.items():
        ref = exp[key]["score"]
        assert abs(s64 - ref) <= 1e-9 * max(1.0, abs(ref)), (key, s64, ref)
        assert model == exp[key]["model"]
        worst = max(worst, abs(s64 - ref))
    kept = O.nms([dict(e, score=got[key][0]) for key, e in exp.items()])
    assert [(int(b["level"]), int(b["i"]), int(b["j"])) for b in boxes[0]] == \
        [(e["level"], e["i"], e["j"]) for e in kept]
    print(f"[rescore all] candidates {len(exp)} equal the oracle's; max |s64 - oracle| {worst:.2e}; "
          f"kept {int(c['kept'])}", flush=True)


def device_candidates(det, frame, w0, h0, sizes):
    cs, ck, _ = det.candidates(frame)
    return [{"score": float(s), "level": int(k[0]), "i": int(k[1]), "j": int(k[2]), "model": int(k[3]),
             "box": O.window_box_q8(w0, h0, *sizes[int(k[0])], int(k[1]), int(k[2]))} for s, k in zip(cs, ck)]


@pytest.mark.parametrize("prec,m", [(pd.PREC_F32, 1), (pd.PREC_BF16, 8)])
def test_overflow_takes_the_highest_scoring(prec, m):
    w0, h0 = 1242, 375
    img = pd_synth.frame(w0, h0, 4600 + m)
    wts, bias = pd_synth.svm_weights(m), np.zeros(m, np.float32)
    levels = O.frame_scores(img, wts, bias, clip=CLIP32, eps=EPS32)
    allmax = np.sort(np.concatenate([O.max_over_models(lv["scores"])[0].ravel() for lv in levels]))
    # FP32: every window is a candidate; BF16: the upper half, the windows
    # within 0.05 of the median rescored in FP64
    thr = -1e30 if prec == pd.PREC_F32 else float(0.5 * (allmax[allmax.size // 2 - 1] + allmax[allmax.size // 2]))
    exp_n = int((allmax > thr).sum())
    assert exp_n > pd.MAX_CANDIDATES
    prm = pd.params(precision=prec)
    print(f"\n[overflow] prec {prec}, {m} models, threshold {thr:.4g}, {exp_n} oracle candidates", flush=True)
    runs = [run([img], wts, bias, [thr], prm) for _ in range(2)]
    det, (boxes, counts) = runs[0]
    c = counts[0]
    assert c["candidates"] == exp_n and c["overflow"] == 1
    sizes = [lv["size"] for lv in levels]
    cands = device_candidates(det, 0, w0, h0, sizes)
    assert len(cands) == exp_n
    exp = {(e["level"], e["i"], e["j"]) for e in O.candidates(levels, w0, h0, thr)}
    assert {(e["level"], e["i"], e["j"]) for e in cands} == exp
    top = O.select_top(cands, pd.MAX_CANDIDATES)
    kept = O.nms(top)
    got = [(int(b["level"]), int(b["i"]), int(b["j"]), int(b["model"])) for b in boxes[0]]
    assert got == [(e["level"], e["i"], e["j"], e["model"]) for e in kept[:1024]]
    assert int(c["kept"]) == min(len(kept), 1024)
    assert boxes[0].tobytes() == runs[1][1][0][0].tobytes() and counts.tobytes() == runs[1][1][1].tobytes()
    print(f"[overflow] {len(cands)} candidates listed, NMS of the top {len(top)} keeps {len(kept)}: equal to the "
          f"oracle's greedy NMS of that selection; two runs bytewise equal", flush=True)


@pytest.mark.parametrize("feat", [pd.FEAT_HOG, pd.FEAT_LBP], ids=["hog", "lbp"])
@pytest.mark.parametrize("m", [1, 3])
def test_bf16_feature_subset(feat, m):
    """BF16 HOG-SVM and LBP-SVM: decisions equal the oracle's with the other
    family's weights at zero, FP64 rescores within 1e-9 of it, and the
    unmasked weights give the same bytes (the other family is never read,
    in the MFMA scoring or in the FP64 rescore)."""
    w0, h0 = 640, 480
    img = pd_synth.frame(w0, h0, 4700 + feat + m)
    raw = pd_synth.svm_weights(m)
    wts = np.array(raw, copy=True)
    if feat == pd.FEAT_HOG:
        wts[:, O.HOG_DIM:] = 0.0
    else:
        wts[:, :O.HOG_DIM] = 0.0
    bias = np.zeros(m, np.float32)
    levels = O.frame_scores(img, wts, bias, clip=CLIP32, eps=EPS32)
    thr = O.frame_threshold(levels)
    prm = pd.params(precision=pd.PREC_BF16, features=feat, margin=0.05)
    det, (boxes, counts) = run([img], wts, bias, [thr], prm)
    _, (boxes_raw, counts_raw) = run([img], raw, bias, [thr], prm)
    exp = {(e["level"], e["i"], e["j"]): e for e in O.candidates(levels, w0, h0, thr)}
    assert counts[0]["overflow"] == 0 and counts[0]["candidates"] == len(exp)
    cs, ck, c64 = det.candidates(0)
    got = {(int(k[0]), int(k[1]), int(k[2])): (float(s), int(k[3]), float(s64)) for s, k, s64 in zip(cs, ck, c64)}
    assert set(got) == set(exp)
    n_res = 0
    for key, (s, model, s64) in got.items():
        ref = exp[key]["score"]
        if not math.isnan(s64):
            n_res += 1
            assert abs(s64 - ref) <= 1e-9 * max(1.0, abs(ref)), (key, s64, ref)
        else:
            assert abs(s - ref) < 0.05, (key, s, ref)
    assert boxes[0].tobytes() == boxes_raw[0].tobytes() and counts.tobytes() == counts_raw.tobytes()
    print(f"\n[bf16 subset] features {feat}, {m} models: candidates {len(exp)} equal the oracle's, "
          f"{int(counts[0]['rescored'])} rescored ({n_res} candidates)", flush=True)


def test_graph_survives_autotune():
    frames = [to_dev(f) for f in pd_synth.frame_batch([(1242, 375), (640, 480)], 4800)]
    wts = to_dev(pd_synth.svm_weights(1))
    bias = to_dev(np.zeros(1, np.float32))
    thr = to_dev(np.array([2.5, 2.5]))
    det = pd.Detector(frames, wts, bias, pd.params(tune_feat_rows=4, tune_score_rows=16), cap=1024)
    det.run(thr)
    torch.cuda.synchronize()
    ref = det.results()
    det.capture(thr)
    det.autotune(thr, iters=1)  # captures and launches graphs of other shapes on the same workspace
    det.replay()
    torch.cuda.synchronize()
    got = det.results()
    for f in range(2):
        assert got[0][f].tobytes() == ref[0][f].tobytes()
    assert got[1].tobytes() == ref[1].tobytes()
    det.release()
