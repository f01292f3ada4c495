"""Pins of the oracle's LBP block histograms (Algorithm 3) and of the
cell-level model that scores windows as a block-level model does, against
definitions independent of the functions under test.  CPU only."""
import numpy as np

import pd_synth
from oracle import pd_oracle as O


def direct_block_histograms(img):
    """Counts of uniform bins over each 16x16 pixel block, straight from the
    per-pixel codes (no cell histograms involved)."""
    h, w = img.shape
    bins = O.uniform_bin_table()[O.lbp_codes(img).astype(np.int64)]
    hb, wb = h // 8 - 1, w // 8 - 1
    out = np.zeros((hb, wb, O.LBP_BINS), np.int64)
    for y in range(hb):
        for x in range(wb):
            out[y, x] = np.bincount(bins[8 * y:8 * y + 16, 8 * x:8 * x + 16].ravel(), minlength=O.LBP_BINS)
    return out


def test_blocks_equal_direct_counts_over_16x16_pixels():
    for w, h, seed in [(64, 48, 1), (83, 57, 2), (160, 136, 3)]:  # ragged edges included
        img = pd_synth.frame(w, h, seed)
        got = O.lbp_block_histograms(O.lbp_cell_histograms(img))
        assert got.shape == (h // 8 - 1, w // 8 - 1, 59)
        assert np.array_equal(got, direct_block_histograms(img))


def test_every_block_counts_256_pixels():
    img = pd_synth.frame(200, 120, 4)
    blocks = O.lbp_block_histograms(O.lbp_cell_histograms(img))
    assert np.all(blocks.sum(axis=2) == 256)
    flat = np.full((40, 40), 7, np.uint8)  # every code is 255 -> bin 57 (uniform, last before 58)
    assert np.all(O.lbp_block_histograms(O.lbp_cell_histograms(flat))[..., 57] == 256)


def test_fold_of_one_block_weight_hits_its_four_cells():
    for (a, b, k) in [(0, 0, 0), (14, 6, 58), (7, 3, 20)]:
        wb = np.zeros((1, O.BLOCK_MODEL_DIM))
        wb[0, O.HOG_DIM + (a * 7 + b) * 59 + k] = 1.0
        wc = O.fold_lbp_block_weights(wb)[0, O.HOG_DIM:].reshape(16, 8, 59)
        expect = np.zeros((16, 8, 59))
        expect[a:a + 2, b:b + 2, k] = 1.0
        assert np.array_equal(wc, expect)
    # HOG weights pass through unchanged
    wb = np.zeros((1, O.BLOCK_MODEL_DIM))
    wb[0, :O.HOG_DIM] = np.arange(O.HOG_DIM)
    assert np.array_equal(O.fold_lbp_block_weights(wb)[0, :O.HOG_DIM], np.arange(O.HOG_DIM))


def test_block_model_scores_equal_folded_cell_model():
    """<block vector, w_b> = <cell vector, fold(w_b)> for every window."""
    img = pd_synth.frame(96, 160, 5)
    hog, cells = O.level_features(img)
    blocks = O.lbp_block_histograms(cells)
    rng = np.random.default_rng(6)
    wb = rng.normal(0.0, 0.01, size=(2, O.BLOCK_MODEL_DIM))
    bias = np.array([0.1, -0.3])
    s_blocks = O.window_scores_blocks(hog, blocks, wb, bias)
    s_cells = O.window_scores(hog, cells, O.fold_lbp_block_weights(wb), bias)
    assert s_blocks.shape == s_cells.shape == (2, 20 - 16 + 1, 12 - 8 + 1)  # windows of 16x8 cells
    assert np.allclose(s_blocks, s_cells, rtol=1e-12, atol=1e-12)


def test_block_window_vector_layout():
    hog = np.zeros((15, 7, 36))
    blocks = np.zeros((15, 7, 59), np.int64)
    blocks[2, 3, 5] = 9
    v = O.window_vector_blocks(hog, blocks, 0, 0)
    assert v.shape == (O.BLOCK_MODEL_DIM,)
    assert v[O.HOG_DIM + (2 * 7 + 3) * 59 + 5] == 9 and v.sum() == 9
