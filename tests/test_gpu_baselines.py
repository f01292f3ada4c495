"""The paper's own kernel mappings (ablation baselines of the px/ns
comparison), through the C ABI, against the FP64 oracle at the same bars as
the library's kernels: LBP histograms bit-exact (Naive and Scalable schemes),
HOG Global within 1e-4 |x| + 1e-6 (with the ramp closed forms), SVM Naive and
warp-level within 1e-4 max(|s|, sigma)."""
import math

import numpy as np
import pytest

import pd_synth
from oracle import pd_oracle as O
from test_gpu_parity import hog_close, scores_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_01642_amd as pd  # noqa: E402

DEV = "cuda:0"
SIZES = [(320, 240), (333, 257), (17, 9), (64, 128), (130, 135), (1242, 375)]


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("w,h", SIZES)
def test_lbp_naive_and_scatter_bit_exact(w, h):
    img = pd_synth.frame(w, h, 610 + w)
    codes = pd.lbp_codes(to_dev(img))
    ref = O.lbp_cell_histograms(img)
    naive = pd.lbp_naive(codes).cpu().numpy()
    scatter = pd.lbp_scatter(codes).cpu().numpy()
    assert naive.shape == scatter.shape == ref.shape
    assert np.array_equal(naive.astype(np.int64), ref)
    assert np.array_equal(scatter.astype(np.int64), ref)
    print(f"\n[baselines] lbp naive/scatter {w}x{h}: bit-exact", flush=True)


@pytest.mark.parametrize("w,h", [s for s in SIZES if s[0] >= 16 and s[1] >= 16])
def test_hog_global_matches_oracle(w, h):
    img = pd_synth.frame(w, h, 620 + w)
    got = pd.hog_global(to_dev(img)).cpu().numpy().transpose(1, 2, 0)
    hog_close(got, O.hog_features(img))


def test_hog_global_closed_forms_and_pitch():
    img = np.tile(np.arange(160, dtype=np.uint8), (64, 1))
    f = pd.hog_global(to_dev(img)).cpu().numpy().transpose(1, 2, 0)[1:-1, 1:-1]
    nzi = [0, 8, 9, 17, 18, 26, 27, 35]
    assert np.allclose(f[..., nzi], 0.2 / math.sqrt(0.320001), rtol=1e-5, atol=0)
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, size=(140, 260), dtype=np.uint8)
    padded = np.zeros((140, 272), np.uint8)
    padded[:, :260] = img
    hog_close(pd.hog_global(to_dev(padded)[:, :260]).cpu().numpy().transpose(1, 2, 0), O.hog_features(img))


@pytest.mark.parametrize("w,h,m", [(64, 128, 1), (333, 257, 3), (640, 480, 1)])
def test_svm_naive_and_wave_on_oracle_features(w, h, m):
    img = pd_synth.frame(w, h, 630 + w)
    hog = O.hog_features(img).astype(np.float32)
    cells = O.lbp_cell_histograms(img).astype(np.uint8)
    wts = pd_synth.svm_weights(m)
    bias = np.linspace(-0.5, 0.5, m).astype(np.float32)
    b, c = to_dev(hog.transpose(2, 0, 1)), to_dev(cells.transpose(2, 0, 1))
    ref = O.window_scores(hog.astype(np.float64), cells, wts, bias)
    for fn in (pd.score_windows_naive, pd.score_windows_wave):
        got = fn(b, c, to_dev(wts), to_dev(bias)).cpu().numpy()
        assert got.shape == ref.shape
        for k in range(m):
            scores_close(got[k], ref[k])
    print(f"\n[baselines] svm naive/wave {w}x{h} m {m}: within 1e-4", flush=True)
