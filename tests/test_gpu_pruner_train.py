"""Training the pruner on the GPU with libpd's own forward/backward kernels,
calibrating its per-frame K for 99 % recall of the plain detector's boxes,
and what the trained network gains over the untrained one."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import pd_synth
from oracle import pd_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_01642_amd as pd  # noqa: E402
from paper_1611_01642_amd import pruner_train as T  # noqa: E402

DEV = "cuda:0"


def frames(seed0, n):
    with ThreadPoolExecutor(16) as ex:
        imgs = list(ex.map(lambda s: pd_synth.frame(1242, 375, s), range(seed0, seed0 + n)))
    return [torch.from_numpy(f).to(DEV) for f in imgs]


def test_trained_pruner_keeps_fewer_windows_at_99_recall():
    wts = torch.from_numpy(pd_synth.svm_weights(1)).to(DEV)
    bias = torch.zeros(1, dtype=torch.float32, device=DEV)
    # detection threshold: the oracle's 99th-percentile rule on a calibration frame
    thr = O.frame_threshold(O.frame_scores(pd_synth.frame(1242, 375, 999), pd_synth.svm_weights(1),
                                           np.zeros(1, np.float32)))
    train_f, cal_f, test_f = frames(20000, 96), frames(30000, 32), frames(40000, 32)
    print(f"\n[train] threshold {thr:.4f}", flush=True)
    data = T.training_set(train_f, wts, bias, thr)
    p0 = torch.from_numpy(pd_synth.pruner_init(seed=11)).to(DEV)
    p, hist, pw = T.train(data, p0, epochs=8, frames_per_step=8, lr=2e-3, seed=1,
                          log=lambda s: print("[train]", s, flush=True))
    print(f"[train] positive weight {pw:.1f}, losses {[round(h, 4) for h in hist]}", flush=True)
    assert np.all(np.isfinite(hist)) and hist[-1] < 0.8 * hist[0]
    thr_cal = torch.full((len(cal_f),), thr, dtype=torch.float64, device=DEV)
    # K is calibrated for 99.5 % recall on the held-out frames, so that frames
    # seen neither in training nor in calibration keep >= 99 %
    k_tr, r_tr, _, n_win = T.calibrate_keep(cal_f, wts, bias, thr_cal, p, 0.995)
    k_0, r_0, _, _ = T.calibrate_keep(cal_f, wts, bias, thr_cal, p0, 0.995)
    print(f"[train] 99.5% recall on held-out frames: trained K {k_tr} ({k_tr / n_win:.1%} of {n_win} windows, "
          f"recall {r_tr:.4f}); untrained K {k_0} ({k_0 / n_win:.1%}, recall {r_0:.4f})", flush=True)
    assert r_tr >= 0.995
    assert k_tr < k_0
    # a third set of frames, at the calibrated K
    thr_test = torch.full((len(test_f),), thr, dtype=torch.float64, device=DEV)
    det = pd.Detector(test_f, wts, bias, pd.params(), cap=1024)
    det.run(thr_test)
    torch.cuda.synchronize()
    plain, _ = det.results()
    r_test, _ = T.recall_at(test_f, wts, bias, thr_test, p, k_tr, plain)
    print(f"[train] recall on unseen frames at K {k_tr}: {r_test:.4f}", flush=True)
    assert r_test >= 0.99


def test_resume_from_checkpoint_is_bitwise(tmp_path):
    """Four epochs straight, against two epochs, a checkpoint, and two more
    epochs resumed from it into fresh buffers: the resumed epochs' losses and
    the final parameters are bitwise the straight run's."""
    wts = torch.from_numpy(pd_synth.svm_weights(1)).to(DEV)
    bias = torch.zeros(1, dtype=torch.float32, device=DEV)
    imgs = [torch.from_numpy(pd_synth.frame(640, 480, s)).to(DEV) for s in range(21000, 21008)]
    data = T.training_set(imgs, wts, bias, 2.5)
    p0 = torch.from_numpy(pd_synth.pruner_init(seed=12)).to(DEV)
    p_a, hist_a, _ = T.train(data, p0, epochs=4, frames_per_step=2, lr=2e-3, seed=5)
    ck = str(tmp_path / "pruner.ckpt")
    _, hist_b1, _ = T.train(data, p0, epochs=2, frames_per_step=2, lr=2e-3, seed=5, checkpoint=ck)
    fresh = torch.full_like(p0, float("nan"))
    p_b, hist_b2, _ = T.train(data, fresh, epochs=4, frames_per_step=2, lr=2e-3, seed=0, resume=ck)
    print(f"\n[resume] straight {hist_a}; first part {hist_b1}; resumed {hist_b2}", flush=True)
    assert hist_b1 == hist_a[:2] and hist_b2 == hist_a[2:]
    assert torch.equal(p_b.view(torch.int32), p_a.view(torch.int32))
    step, seed = pd.pruner_load(ck, torch.empty_like(p0))
    assert (step, seed) == (8, 5)
