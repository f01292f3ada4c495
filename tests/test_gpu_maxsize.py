"""Parity at the largest accepted image side (PD_MAX_DIM = 16384).

At that side level 0 has 2048 cells per row, so window anchors reach cell
column 2040 and cell row 2032, the widest indices the candidate keys and the
NMS sort key carry.  Two frames that are long in one direction only
(16384x136, one level; 72x16384, two levels) are small enough for the FP64
oracle, which checks them exactly as the full-size tests do (candidate sets,
scores to the FP32 bound, the kept list).  The 16384x16384 frame (51 levels,
about 24 million windows) is checked on sampled candidates: a window's
features depend only on the pixels of the window and a one-pixel ring around
it, so the oracle scores a sampled window from a crop of its level that keeps
an 8-pixel (one-cell) margin wherever the level extends past the window."""
import numpy as np
import pytest

import pd_synth
from oracle import pd_oracle as O
from oracle import pruner_oracle as P
from test_gpu_fullsize import BENCH_TUNING, check_valid_nms, compare_frame, run_graph
from test_gpu_pruned_detect import gpu_keep

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_01642_amd as pd  # noqa: E402

CELL = 8
# the library's L2-Hys parameters are FP32; FP64 rescores are compared with the oracle run on their values
CLIP32, EPS32 = float(np.float32(0.2)), float(np.float32(1e-3))


def test_longest_sides_match_oracle():
    # the first two take their own 99th-percentile thresholds; the last two,
    # one window row or column, take every window as a candidate (2041 and
    # 2033 of them, within the list's capacity), so the farthest anchors
    # (column 2040, row 2032) go through compaction, the sort and NMS
    sizes = [(16384, 136), (72, 16384), (16384, 128), (64, 16384)]
    frames = [pd_synth.frame(w, h, 7000 + k) for k, (w, h) in enumerate(sizes)]
    wts, bias = pd_synth.svm_weights(1), pd_synth.svm_bias(1)
    thr = [O.detect(f, wts, bias)[1] for f in frames[:2]] + [-1e30, -1e30]
    print(f"\n[maxsize] frames {sizes}, thresholds {thr}", flush=True)
    (boxes, counts), det = run_graph(frames, wts, bias, thr, pd.params(**BENCH_TUNING))
    for f, (w, h) in enumerate(sizes):
        check_valid_nms(boxes[f])
        nc, nk = compare_frame(det, f, boxes[f], counts[f], frames[f], wts, bias, thr[f])
        _, ck, _ = det.candidates(f)
        reach = int(ck[:, 2].max()) if w > h else int(ck[:, 1].max())
        if f >= 2:
            assert nc == (2041 if w > h else 2033) and reach == (2040 if w > h else 2032)
        print(f"[maxsize] {w}x{h}: candidates {nc}, kept {nk} equal the oracle's; farthest anchor {reach}",
              flush=True)


def crop_score(level, i, j, wts, bias):
    """FP64 oracle score of the window anchored at cell (i, j) of `level`,
    from a crop with a one-cell margin where the level has one."""
    h, w = level.shape
    y0, x0 = max(0, CELL * (i - 1)), max(0, CELL * (j - 1))
    y1 = min(h, CELL * (i + O.WIN_CELLS_Y + 1))
    x1 = min(w, CELL * (j + O.WIN_CELLS_X + 1))
    hog, cells = O.level_features(level[y0:y1, x0:x1])
    v = O.window_vector(hog, cells, i - y0 // CELL, j - x0 // CELL)
    return float(v @ wts[0].astype(np.float64) + float(bias[0]))


def test_largest_frame_sampled_candidates():
    W = H = 16384
    # a seeded 2048x2048 frame tiled 8 x 8 (generating the full frame directly
    # takes about a minute on the host)
    frame = np.ascontiguousarray(np.tile(pd_synth.frame(2048, 2048, 7100), (8, 8)))
    wts, bias = pd_synth.svm_weights(1), pd_synth.svm_bias(1)
    # threshold: the highest window score of a 1242x375 frame, so that about one
    # window in 18,000 passes and the candidate list stays within its capacity
    thr = max(float(lv["scores"].max()) for lv in O.frame_scores(pd_synth.frame(1242, 375, 1000), wts, bias))
    sizes = O.level_sizes(W, H)
    print(f"\n[maxsize] {W}x{H}, {len(sizes)} levels, threshold {thr:.6f}", flush=True)
    (boxes, counts), det = run_graph([frame], wts, bias, [thr], pd.params(**BENCH_TUNING))
    c, cap = counts[0], 1024
    check_valid_nms(boxes[0])
    cs, ck, _ = det.candidates(0)
    n = int(c["candidates"])
    assert len(cs) == n > 0  # the list holds every candidate
    # the kept list is the oracle's greedy NMS of the PD_MAX_CANDIDATES
    # highest-scoring candidates (all of them when there are no more; on the
    # device's FP32 scores, as in the full-size tests), truncated to the
    # capacity; overflow says whether either limit was reached
    cand = [{"score": float(s), "level": int(k[0]), "i": int(k[1]), "j": int(k[2]),
             "box": O.window_box_q8(W, H, *sizes[int(k[0])], int(k[1]), int(k[2]))} for s, k in zip(cs, ck)]
    kept = O.nms(O.select_top(cand, pd.MAX_CANDIDATES))
    assert int(c["kept"]) == min(len(kept), cap)
    assert c["overflow"] == int(len(kept) > cap or n > pd.MAX_CANDIDATES)
    assert [(int(b["level"]), int(b["i"]), int(b["j"])) for b in boxes[0]] == \
        [(k["level"], k["i"], k["j"]) for k in kept[:cap]]
    for b, k in zip(boxes[0], kept):
        assert (b["x0"], b["y0"], b["x1"], b["y1"]) == k["box"]
    for s, k in zip(cs, ck):
        lw, lh = sizes[int(k[0])]
        ny, nx = O.window_grid(lw, lh)
        assert 0 <= k[1] < ny and 0 <= k[2] < nx and k[3] == 0
        assert float(s) > thr - 1e-4 * max(abs(thr), 1.0)
    # sampled: at level 0 (the frame itself) the farthest anchors in each
    # direction and a few seeded others; at the small levels, one each
    rng = np.random.default_rng(7101)
    l0 = np.flatnonzero(ck[:, 0] == 0)
    pick = set()
    if len(l0):
        pick |= {int(l0[np.argmax(ck[l0, 1])]), int(l0[np.argmax(ck[l0, 2])]), int(l0[np.argmin(ck[l0, 2])])}
        pick |= {int(q) for q in rng.choice(l0, size=min(4, len(l0)), replace=False)}
    small = [q for q in range(len(ck)) if sizes[int(ck[q, 0])][0] <= 2048]
    by_level = {}
    for q in small:
        by_level.setdefault(int(ck[q, 0]), q)
    pick |= set(list(by_level.values())[:4])
    assert pick
    for q in sorted(pick):
        lvl, i, j = int(ck[q, 0]), int(ck[q, 1]), int(ck[q, 2])
        level = frame if lvl == 0 else O.resize(frame, *sizes[lvl])
        ref = crop_score(level, i, j, wts, bias)
        assert abs(float(cs[q]) - ref) <= 1e-4 * max(abs(ref), 1.0), (lvl, i, j, float(cs[q]), ref)
        assert ref > thr - 1e-4 * max(abs(thr), 1.0)
    print(f"[maxsize] candidates {int(c['candidates'])}, kept {int(c['kept'])}; {len(pick)} sampled scores "
          f"({len(l0)} level-0 candidates, anchors to row {int(ck[l0, 1].max()) if len(l0) else -1}, "
          f"column {int(ck[l0, 2].max()) if len(l0) else -1}) equal the oracle's", flush=True)


@pytest.mark.parametrize("m", [1, 8])
def test_bf16_longest_sides_decisions(m):
    """BF16 MFMA scoring with FP64 rescoring at the largest side: the
    candidate sets equal the oracle's, rescored windows carry its FP64 score
    within 1e-9 (clip and eps as their FP32 values, which the library uses)
    and the others are within the rescoring margin."""
    sizes = [(16384, 136), (72, 16384), (16384, 128), (64, 16384)]
    frames = [pd_synth.frame(w, h, 7200 + k) for k, (w, h) in enumerate(sizes)]
    wts, bias = pd_synth.svm_weights(m), np.zeros(m, np.float32)
    levels = [O.frame_scores(f, wts, bias, clip=CLIP32, eps=EPS32) for f in frames]
    thr = [O.frame_threshold(lv) for lv in levels[:2]] + [-1e30, -1e30]
    prm = pd.params(precision=pd.PREC_BF16, margin=0.05, tune_feat_rows=12, tune_grid=0)
    (boxes, counts), det = run_graph(frames, wts, bias, thr, prm)
    for f, (w, h) in enumerate(sizes):
        assert counts[f]["overflow"] == 0
        check_valid_nms(boxes[f])
        exp = {(c["level"], c["i"], c["j"]): c for c in O.candidates(levels[f], w, h, thr[f])}
        cs, ck, c64 = det.candidates(f)
        got = {(int(k[0]), int(k[1]), int(k[2])): (float(s), int(k[3]), float(s64))
               for s, k, s64 in zip(cs, ck, c64)}
        assert set(got) == set(exp)
        n_res = 0
        for key, (s, model, s64) in got.items():
            ref = exp[key]["score"]
            if not np.isnan(s64):
                n_res += 1
                assert abs(s64 - ref) <= 1e-9 * max(1.0, abs(ref)), (key, s64, ref)
                assert model == exp[key]["model"]
            else:
                assert abs(s - ref) < 0.05, (key, s, ref)
        print(f"\n[maxsize bf16] {w}x{h}, {m} models: candidates {len(exp)} equal the oracle's, {n_res} rescored",
              flush=True)


def test_pruned_longest_sides():
    """The pruner at the largest side: BF16 logits against the FP64 network
    on the oracle's cell map, and pruned detection (keep set from the device's
    logits and the top-K rule, as in the pruned-detection tests) equal to the
    oracle's detections restricted to the kept windows."""
    sizes = [(16384, 136), (72, 16384)]
    frames = [pd_synth.frame(w, h, 7300 + k) for k, (w, h) in enumerate(sizes)]
    params = pd_synth.pruner_init(seed=7301)
    pr = torch.from_numpy(params).to("cuda:0")
    wts, bias = pd_synth.svm_weights(1), np.zeros(1, np.float32)
    for f, (w, h) in enumerate(sizes):
        img = frames[f]
        got = pd.pruner_logits_bf16(torch.from_numpy(img).to("cuda:0"), pr).cpu().numpy().astype(np.float64)
        exp, _ = P.forward(P.cellmap(img), params.astype(np.float64))
        scale = np.abs(exp).max()
        assert got.shape == exp.shape and np.abs(got - exp).max() <= 2e-2 * scale
        levels = O.frame_scores(img, wts, bias)
        thr = O.frame_threshold(levels)
        n_win = sum(lv["scores"][0].size for lv in levels)
        k = n_win // 2
        prm = pd.params(prune_keep=k, pruner=pr)
        keep, _ = gpu_keep(img, pr, k, prm)
        assert sum(int(x.sum()) for x in keep) >= k
        exp_c = [c for c in O.candidates(levels, w, h, thr) if keep[c["level"]][c["i"], c["j"]]]
        det = pd.Detector([torch.from_numpy(img).to("cuda:0")], torch.from_numpy(wts).to("cuda:0"),
                          torch.from_numpy(bias).to("cuda:0"), prm, cap=1024)
        det.run(torch.tensor([thr], dtype=torch.float64, device="cuda:0"))
        torch.cuda.synchronize()
        boxes, counts = det.results()
        _, ck, _ = det.candidates(0)
        assert counts[0]["overflow"] == 0
        assert {(int(a[0]), int(a[1]), int(a[2])) for a in ck} == {(c["level"], c["i"], c["j"]) for c in exp_c}
        assert [(int(b["level"]), int(b["i"]), int(b["j"])) for b in boxes[0]] == \
            [(c["level"], c["i"], c["j"]) for c in O.nms(exp_c)]
        print(f"\n[maxsize pruned] {w}x{h}: logits within {np.abs(got - exp).max() / scale:.2g} of the scale; "
              f"K {k} of {n_win}, candidates {len(exp_c)} equal the oracle's", flush=True)
