"""The detection context (pd_ctx_*): its graph cache and its tuning table.

* pd_ctx_detect replays a cached graph for repeated calls on the same
  arguments; with new pixels written into the same frame buffers and new
  thresholds between calls, every call equals an eager pd_detect on the same
  inputs, byte for byte.
* More argument sets than the cache holds (8): the least recently used graph
  is released and recaptured when needed; results stay exact.
* pd_ctx_autotune stores its choice: a second call returns it without
  timing, and pd_ctx_detect with default tuning fields uses it (same bytes as
  pd_detect with those fields).
"""
import time

import numpy as np
import pytest

import pd_synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_01642_amd as pd  # noqa: E402

DEV = "cuda:0"
SIZES = [(1242, 375), (640, 480)]


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def eager(frames, wts, bias, prm, thr):
    det = pd.Detector(frames, wts, bias, prm, cap=512)
    det.run(thr)
    torch.cuda.synchronize()
    return det.results()


def same(a, b):
    assert a[1].tobytes() == b[1].tobytes()
    for f in range(len(a[0])):
        assert a[0][f].tobytes() == b[0][f].tobytes(), f


@pytest.mark.parametrize("prec,m", [(pd.PREC_F32, 1), (pd.PREC_BF16, 4)])
def test_ctx_detect_replays_equal_eager(prec, m):
    ctx = pd.Context()
    frames = [to_dev(f) for f in pd_synth.frame_batch(SIZES, 9000)]
    wts = to_dev(pd_synth.svm_weights(m))
    bias = to_dev(np.zeros(m, np.float32))
    thr = to_dev(np.full(2, 2.5 if m == 1 else 5.0))
    prm = pd.params(precision=prec)
    det = pd.Detector(frames, wts, bias, prm, cap=512, ctx=ctx)
    for rep in range(4):
        new = pd_synth.frame_batch(SIZES, 9100 + rep)
        for dst, src in zip(frames, new):
            dst.copy_(to_dev(src))
        thr.fill_(2.5 + 0.1 * rep if m == 1 else 5.0 + 0.2 * rep)
        det.run(thr)
        torch.cuda.synchronize()
        got = det.results()
        assert all(c["candidates"] > 0 for c in got[1])
        same(got, eager(frames, wts, bias, prm, thr))
        print(f"\n[ctx] prec {prec} models {m} call {rep}: equals eager pd_detect", flush=True)
    ctx.close()


def test_ctx_graph_cache_eviction():
    ctx = pd.Context()
    frames = [to_dev(pd_synth.frame(640, 480, 9200))]
    wts = to_dev(pd_synth.svm_weights(1))
    bias = to_dev(np.zeros(1, np.float32))
    det = pd.Detector(frames, wts, bias, pd.params(), cap=512, ctx=ctx)
    thrs = [to_dev(np.array([1.5 + 0.1 * k])) for k in range(11)]  # 11 buffers: 11 argument sets
    for rnd in range(2):
        for k, t in enumerate(thrs):
            det.run(t)
            torch.cuda.synchronize()
            same(det.results(), eager(frames, wts, bias, pd.params(), t))
    ctx.close()


def test_ctx_autotune_is_remembered(tmp_path):
    ctx = pd.Context()
    frames = [to_dev(f) for f in pd_synth.frame_batch(SIZES, 9300)]
    wts = to_dev(pd_synth.svm_weights(1))
    bias = to_dev(np.zeros(1, np.float32))
    thr = to_dev(np.full(2, 2.5))
    det = pd.Detector(frames, wts, bias, pd.params(), cap=512, ctx=ctx)
    t0 = time.perf_counter()
    tuning, ms = det.autotune(thr, iters=1)
    t1 = time.perf_counter()
    det.prm = pd.params()
    tuning2, ms2 = det.autotune(thr, iters=1)
    t2 = time.perf_counter()
    assert tuning2 == tuning and ms2 == ms
    assert t2 - t1 < 0.1 * (t1 - t0)
    print(f"\n[ctx] autotune {tuning} ({ms:.3f} ms/call) in {t1 - t0:.2f} s, remembered in {t2 - t1:.4f} s",
          flush=True)
    assert ctx.tuning(SIZES, 1, pd.params()).tuning() == tuning
    det.prm = pd.params()  # default fields: the context applies its entry
    det.run(thr)
    torch.cuda.synchronize()
    same(det.results(), eager(frames, wts, bias, pd.params(**tuning), thr))
    path = str(tmp_path / "tuning.txt")
    ctx.save(path)
    other = pd.Context()
    other.load(path)
    assert other.tuning(SIZES, 1, pd.params()).tuning() == tuning
    other.close()
    ctx.close()
