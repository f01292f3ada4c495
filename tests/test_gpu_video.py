"""Streaming video mode (pd_video_*): frames pushed from host memory come
back, in push order, with exactly the boxes and counts pd_detect gives for
each frame on its own (the same kernels, replayed from per-slot graphs),
across ring wrap-around and pitched host frames."""
import numpy as np
import pytest

import pd_synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_01642_amd as pd  # noqa: E402

DEV = "cuda:0"


def reference(frames, wts, bias, thr):
    out = []
    for f, t in zip(frames, thr):
        det = pd.Detector([torch.from_numpy(f).to(DEV)], wts, bias, pd.params(), cap=256)
        det.run(torch.tensor([t], dtype=torch.float64, device=DEV))
        torch.cuda.synchronize()
        boxes, counts = det.results()
        out.append((boxes[0], counts[0]))
    return out


@pytest.mark.parametrize("w,h,depth,n", [(640, 480, 3, 7), (1242, 375, 2, 7), (333, 257, 1, 7), (640, 480, 16, 21),
                                         (65, 129, 4, 9)])
def test_video_equals_per_frame_detect(w, h, depth, n):
    """Depth 16 is the largest ring; a 65x129 frame has exactly one window,
    which every frame reports (threshold below any score)."""
    print(f"video {w}x{h} depth {depth}", flush=True)
    frames = [pd_synth.frame(w, h, 1500 + k) for k in range(n)]
    one_window = (w // 8 - 7) * (h // 8 - 15) == 1
    if one_window:
        thr = [-1e30] * n
    else:
        thr = [4.0 + 0.4 * (k % 3) for k in range(n)]  # a few hundred candidates, below the list cap
    wts = torch.from_numpy(pd_synth.svm_weights(1)).to(DEV)
    bias = torch.from_numpy(pd_synth.svm_bias(1)).to(DEV)
    ref = reference(frames, wts, bias, thr)
    v = pd.Video(w, h, wts, bias, cap=256, depth=depth)
    got, k = [], 0
    while len(got) < len(frames):  # keep the ring full, pop the oldest: wraps around
        while k < len(frames) and k - len(got) < depth:
            v.push(frames[k], thr[k])
            k += 1
        got.append(v.pop())
    v.close()
    assert len(got) == len(frames)
    for (gb, gc, ms), (rb, rc) in zip(got, ref):
        assert rc["overflow"] == 0 and rc["kept"] > 0
        if one_window:
            assert rc["candidates"] == 1 and rc["kept"] == 1
        assert gb.tobytes() == rb.tobytes()
        assert gc.tobytes() == rc.tobytes()
        assert ms > 0.0


def test_video_pitched_frames_and_ring_errors():
    w, h = 400, 300
    wide = [np.zeros((h, 448), np.uint8) for _ in range(3)]
    for k, a in enumerate(wide):
        a[:, :w] = pd_synth.frame(w, h, 1600 + k)
    wts = torch.from_numpy(pd_synth.svm_weights(2)).to(DEV)
    bias = torch.zeros(2, device=DEV)
    ref = reference([np.ascontiguousarray(a[:, :w]) for a in wide], wts, bias, [4.0] * 3)
    v = pd.Video(w, h, wts, bias, cap=256, depth=2)
    with pytest.raises(pd.PdError):
        v.pop()  # nothing in flight
    v.push(wide[0][:, :w], 4.0)
    v.push(wide[1][:, :w], 4.0)
    with pytest.raises(pd.PdError):
        v.push(wide[2][:, :w], 4.0)  # both slots in flight
    got = [v.pop()]
    v.push(wide[2][:, :w], 4.0)
    got += [v.pop(), v.pop()]
    v.close()
    for (gb, gc, _), (rb, rc) in zip(got, ref):
        assert gb.tobytes() == rb.tobytes() and gc.tobytes() == rc.tobytes()
