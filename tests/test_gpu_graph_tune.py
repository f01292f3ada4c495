"""Tile-shape tuning, the autotuner and HIP-graph replay of pd_detect.

The tuning fields of pd_params change only how the work is partitioned, so
every tuned run must give the default run's boxes and counts byte for byte.
A captured graph is replayed several times with new pixels written into the
same frame buffers and new thresholds, with other eager work in between;
every replay must equal an eager pd_detect on the same inputs.
"""
import ctypes

import numpy as np
import pytest

import pd_synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_01642_amd as pd  # noqa: E402

DEV = "cuda:0"
SIZES = [(1242, 375), (640, 480), (320, 240)]


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _frames(seed):
    return [to_dev(f) for f in pd_synth.frame_batch(SIZES, seed)]


def _run(frames, wts, bias, prm, thr):
    det = pd.Detector(frames, wts, bias, prm, cap=1024)
    det.run(thr)
    torch.cuda.synchronize()
    return det.results()


def _same(a, b):
    (ba, ca), (bb, cb) = a, b
    assert ca.tobytes() == cb.tobytes(), (ca, cb)
    for f in range(len(ba)):
        assert ba[f].tobytes() == bb[f].tobytes(), f


@pytest.mark.parametrize("prec,m", [(pd.PREC_F32, 2), (pd.PREC_BF16, 1), (pd.PREC_BF16, 4)])
def test_tuning_fields_keep_results(prec, m):
    frames = _frames(5000)
    wts = to_dev(pd_synth.svm_weights(m))
    bias = to_dev(np.zeros(m, np.float32))
    # thresholds that keep every frame's candidates within what NMS takes whole
    thr = to_dev(np.full(3, {1: 2.5, 2: 4.0, 4: 8.0}[m]))
    ref = _run(frames, wts, bias, pd.params(precision=prec), thr)
    assert all(c["candidates"] > 0 and c["overflow"] == 0 for c in ref[1])
    shapes = [dict(tune_feat_rows=4), dict(tune_feat_rows=6), dict(tune_feat_rows=13), dict(tune_feat_rows=32),
              dict(tune_grid=7), dict(tune_grid=300), dict(tune_feat_rows=12, tune_grid=1)]
    if prec == pd.PREC_F32:
        shapes += [dict(tune_score_rows=16), dict(tune_score_rows=16, tune_grid=5), dict(tune_score_rows=4),
                   dict(tune_score_rows=4, tune_grid=3)]
    for kw in shapes:
        print(f"\n[tuning] prec {prec} models {m} {kw}", flush=True)
        _same(ref, _run(frames, wts, bias, pd.params(precision=prec, **kw), thr))


def test_workspace_independent_of_tuning():
    a = pd.workspace_bytes(SIZES, 3, pd.params())
    b = pd.workspace_bytes(SIZES, 3, pd.params(tune_feat_rows=4, tune_score_rows=16, tune_grid=64))
    assert a == b


@pytest.mark.parametrize("prec,m", [(pd.PREC_F32, 1), (pd.PREC_BF16, 8)])
def test_graph_replays_equal_eager(prec, m):
    frames = _frames(6000)
    wts = to_dev(pd_synth.svm_weights(m))
    bias = to_dev(np.zeros(m, np.float32))
    prm = pd.params(precision=prec)
    thr = to_dev(np.full(3, 10.0 if m > 1 else 2.5))
    g = pd.Detector(frames, wts, bias, prm, cap=1024)
    g.capture(thr)
    other = _frames(6500)
    for rep in range(4):
        new = _frames(7000 + 10 * rep)
        for dst, src in zip(frames, new):
            dst.copy_(src)
        thr.copy_(thr + 0.1 * rep)
        print(f"\n[graph] prec {prec} models {m} replay {rep}", flush=True)
        g.replay()
        # unrelated eager work on the same stream between replays
        _run(other, wts, bias, prm, thr)
        torch.cuda.synchronize()
        got = g.results()
        exp = _run([f.clone() for f in frames], wts, bias, prm, thr)
        assert all(c["overflow"] == 0 for c in exp[1])
        _same(exp, got)
        assert sum(int(c["kept"]) for c in got[1]) > 0
    g.release()


def test_graph_stage_events_per_capture():
    """Captures taken while stage profiling is on carry their own stage clock
    stamps: replayed back to back, each reports its own stage times (upload
    about 0: a graph copies nothing; the others positive), and the replays'
    result equals eager pd_detect."""
    frames = _frames(8000)
    wts = to_dev(pd_synth.svm_weights(1))
    bias = to_dev(np.zeros(1, np.float32))
    thr = to_dev(np.full(3, 2.5))
    prm = pd.params()
    det = pd.Detector(frames, wts, bias, prm, cap=1024)
    pd.profile_enable(True)
    try:
        det.capture_steps(thr, 3)
    finally:
        pd.profile_enable(False)
    exp = _run(frames, wts, bias, prm, thr)
    for k in range(3):
        print(f"\n[graph stages] replay {k}", flush=True)
        det.replay_step(k)
    torch.cuda.synchronize()
    for k in range(3):
        st = det.step_stage_ms(k)
        print(f"[graph stages] capture {k}: {st}", flush=True)
        assert 0.0 <= st["upload"] < 0.05
        assert all(st[q] > 0.0 for q in ("resize", "features", "score", "compact", "nms"))
        assert sum(st.values()) < 1000.0
    _same(exp, det.results())
    det.release()
    # a capture without profiling has no stage stamps
    det.capture(thr)
    with pytest.raises(pd.PdError):
        pd._check(pd.lib().pd_graph_stage_ms(det._graph, (ctypes.c_double * len(pd.STAGES))()))
    det.release()


def test_autotune_gives_valid_fields_and_same_results():
    frames = _frames(5000)
    wts = to_dev(pd_synth.svm_weights(2))
    bias = to_dev(np.zeros(2, np.float32))
    thr = to_dev(np.array([4.0, 4.0, 4.0]))  # no candidate list overflows on these frames
    prm = pd.params()
    det = pd.Detector(frames, wts, bias, prm, cap=1024)
    tuning, ms = det.autotune(thr, iters=2)
    print(f"\n[autotune] {tuning} {ms:.3f} ms", flush=True)
    assert tuning["tune_feat_rows"] in (4, 6, 8, 10, 12, 14, 16)
    assert tuning["tune_score_rows"] in (4, 8, 16)
    assert tuning["tune_grid"] in (0, 256, 512, 1024, 2048)
    assert 0.0 < ms < 1000.0
    det.run(thr)
    torch.cuda.synchronize()
    ref = _run(frames, wts, bias, pd.params(), thr)
    assert all(c["overflow"] == 0 for c in ref[1])
    _same(ref, det.results())
