"""pd_detect with learned pruning against the FP64 oracle.

The keep decision (logit >= the frame's K-th largest window logit) is an
integer decision taken from floating point; both sides take it from the same
BF16-inference logits (read back through pd_pruner_logits_bf16, the same
kernels pd_detect runs).  Given that keep set, candidates and kept boxes
must equal the oracle's detections restricted to the kept windows."""
import numpy as np
import pytest

import pd_synth
from oracle import pd_oracle as O
from oracle import pruner_oracle as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_01642_amd as pd  # noqa: E402

DEV = "cuda:0"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gpu_keep(img, pruner_dev, k, prm):
    """Per-level keep masks from the GPU's logits and the top-K rule."""
    _, _, views = pd.build_pyramid(to_dev(img), prm)
    zl = []
    for v in views:
        z = pd.pruner_logits_bf16(v.contiguous(), pruner_dev, prm).cpu().numpy()
        hc, wc = z.shape
        zl.append(P.window_logits(z, hc - 15, wc - 7))
    return P.keep_topk(zl, k), zl


def run(frames, wts, bias, thr, prm, cap=1024):
    det = pd.Detector([to_dev(f) for f in frames], to_dev(wts), to_dev(bias), prm, cap=cap)
    det.run(to_dev(np.asarray(thr, np.float64)))
    torch.cuda.synchronize()
    return det


@pytest.mark.parametrize("prec,m,k", [(pd.PREC_F32, 1, 3000), (pd.PREC_F32, 1, 150), (pd.PREC_BF16, 1, 3000),
                                      (pd.PREC_BF16, 4, 6000)])
def test_pruned_detect_equals_oracle_on_kept_windows(prec, m, k):
    img = pd_synth.frame(1242, 375, 1000)
    wts, bias = pd_synth.svm_weights(m), np.zeros(m, np.float32)
    levels = O.frame_scores(img, wts, bias, 11, 10, 0)
    thr = O.frame_threshold(levels)
    pr = to_dev(pd_synth.pruner_init(seed=5))
    prm = pd.params(precision=prec, prune_keep=k, pruner=pr)
    keep, _ = gpu_keep(img, pr, k, prm)
    n_keep = sum(int(x.sum()) for x in keep)
    assert n_keep >= k
    print(f"\n[pruned] prec {prec} models {m} K {k}: {n_keep} of {sum(x.size for x in keep)} windows kept", flush=True)
    exp = [c for c in O.candidates(levels, 1242, 375, thr) if keep[c["level"]][c["i"], c["j"]]]
    det = run([img], wts, bias, [thr], prm)
    boxes, counts = det.results()
    cs, ck, c64 = det.candidates(0)
    got = {(int(a[0]), int(a[1]), int(a[2])) for a in ck}
    assert counts[0]["overflow"] == 0
    assert got == {(c["level"], c["i"], c["j"]) for c in exp}
    kept = O.nms(exp)
    assert [(int(b["level"]), int(b["i"]), int(b["j"])) for b in boxes[0]] == \
        [(c["level"], c["i"], c["j"]) for c in kept]


def test_keeping_every_window_equals_plain_detect():
    frames = pd_synth.frame_batch([(640, 480), (1242, 375)], 4000)
    wts, bias = pd_synth.svm_weights(2), np.zeros(2, np.float32)
    pr = to_dev(pd_synth.pruner_init(seed=6))
    thr = [4.0, 4.0]
    plain = run(frames, wts, bias, thr, pd.params()).results()
    pruned = run(frames, wts, bias, thr, pd.params(prune_keep=10 ** 6, pruner=pr)).results()
    assert plain[1].tobytes() == pruned[1].tobytes()
    for a, b in zip(plain[0], pruned[0]):
        assert a.tobytes() == b.tobytes()


def test_pruned_batch_equals_single_frames():
    frames = pd_synth.frame_batch([(1242, 375), (640, 480), (1242, 375)], 4100)
    wts, bias = pd_synth.svm_weights(1), np.zeros(1, np.float32)
    pr = to_dev(pd_synth.pruner_init(seed=7))
    prm = pd.params(precision=pd.PREC_BF16, prune_keep=2000, pruner=pr)
    thr = [3.0, 3.0, 3.0]
    batch = run(frames, wts, bias, thr, prm).results()
    for f in range(3):
        single = run([frames[f]], wts, bias, thr[:1], prm).results()
        b = batch[0][f].copy()
        b["frame"] = 0
        assert b.tobytes() == single[0][0].tobytes()
        assert batch[1][f]["candidates"] == single[1][0]["candidates"]
