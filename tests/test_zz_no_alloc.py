"""pd_detect_noalloc (the static-scratch variant of pd_detect) against
pd_detect, through the C ABI: boxes and counts byte for byte on two calls in
a row, the second with a smaller batch, then a BF16 call; a batch beyond the
scratch is rejected before any GPU work."""
import numpy as np
import pytest

import pd_synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_01642_amd as pd  # noqa: E402

DEV = "cuda:0"
CAP = 512


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def both(frames, wts, bias, prm, thr):
    det = pd.Detector(frames, wts, bias, prm, cap=CAP)
    det.run(thr)
    n = len(frames)
    boxes = torch.zeros(n * CAP * pd.BOX_DTYPE.itemsize, dtype=torch.uint8, device=DEV)
    counts = torch.zeros(n * pd.COUNTS_DTYPE.itemsize, dtype=torch.uint8, device=DEV)
    pd.detect_noalloc(frames, wts, bias, prm, thr, boxes, counts, CAP)
    torch.cuda.synchronize()
    return (det.boxes.cpu().numpy(), det.counts.cpu().numpy()), (boxes.cpu().numpy(), counts.cpu().numpy())


def check_equal(ref, got, n):
    (rb, rc), (gb, gc) = ref, got
    assert rc.tobytes() == gc.tobytes()
    counts = rc.view(pd.COUNTS_DTYPE)
    rbx = rb.view(pd.BOX_DTYPE).reshape(n, CAP)
    gbx = gb.view(pd.BOX_DTYPE).reshape(n, CAP)
    for f in range(n):
        k = int(counts[f]["kept"])
        assert k > 0 and counts[f]["overflow"] == 0
        assert rbx[f, :k].tobytes() == gbx[f, :k].tobytes(), f
    return int(counts["candidates"].sum()), int(counts["kept"].sum())


def test_noalloc_equals_detect():
    wts1, bias1 = to_dev(pd_synth.svm_weights(1)), to_dev(np.zeros(1, np.float32))
    big = [to_dev(f) for f in pd_synth.frame_batch([(1242, 375), (1242, 375), (640, 480)], 8100)]
    print("\n[noalloc] call 1: 2 x 1242x375 + 640x480, FP32", flush=True)
    ref, got = both(big, wts1, bias1, pd.params(), to_dev(np.array([2.5, 2.5, 2.5])))
    print("[noalloc] call 1 candidates / kept:", check_equal(ref, got, 3), flush=True)
    small = [to_dev(pd_synth.frame(320, 240, 8200))]
    print("[noalloc] call 2: one 320x240 frame, FP32, scale 6/5, 3 levels", flush=True)
    prm = pd.params(scale=(6, 5), max_levels=3)
    ref, got = both(small, wts1, bias1, prm, to_dev(np.array([1.0])))
    print("[noalloc] call 2 candidates / kept:", check_equal(ref, got, 1), flush=True)
    wts8, bias8 = to_dev(pd_synth.svm_weights(8)), to_dev(np.zeros(8, np.float32))
    print("[noalloc] call 3: 1242x375, BF16, 8 models", flush=True)
    ref, got = both([big[0]], wts8, bias8, pd.params(precision=pd.PREC_BF16), to_dev(np.array([6.3])))
    print("[noalloc] call 3 candidates / kept:", check_equal(ref, got, 1), flush=True)


def test_noalloc_rejects_oversize_batch():
    frames = [to_dev(pd_synth.frame(1920, 1080, 8300))] * 2
    assert pd.workspace_bytes([(1920, 1080)] * 2) > pd.NOALLOC_SCRATCH_BYTES
    wts1, bias1 = to_dev(pd_synth.svm_weights(1)), to_dev(np.zeros(1, np.float32))
    boxes = torch.zeros(2 * CAP * pd.BOX_DTYPE.itemsize, dtype=torch.uint8, device=DEV)
    counts = torch.zeros(2 * pd.COUNTS_DTYPE.itemsize, dtype=torch.uint8, device=DEV)
    with pytest.raises(pd.PdError) as e:
        pd.detect_noalloc(frames, wts1, bias1, pd.params(), to_dev(np.array([2.5, 2.5])), boxes, counts, CAP)
    assert e.value.code == pd.E_WORKSPACE
