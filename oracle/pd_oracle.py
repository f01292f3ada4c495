"""Plain FP64 CPU oracle for the HOG+LBP+SVM detection hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares no code with
the HIP path (no kernels, headers, tables or helpers); both sides read their
inputs from the seeded generator package `pd_synth`.

Everything here is the literal definition of each result, in float64 unless
the quantity is an integer, written for readability rather than speed:
  * pyramid levels       -- Section 4.4 (pyramidal sliding window) and
                            Section 4.1 step (2); fixed-point bilinear resize
  * LBP codes            -- Section 4.2, Algorithm 1
  * LBP cell histograms  -- Section 4.2, Algorithm 2 (uniform 59-bin LUT)
  * gradients            -- Section 4.3, Algorithm 4
  * HOG block histograms -- Section 4.3, Algorithm 5 (per block, every pixel
                            of the 16x16 block votes with trilinear weights)
  * L2-Hys normalisation -- block normalisation of the HOG descriptor
                            (Dalal and Triggs, cited in Section 4.3)
  * window scores        -- Section 4.4, Algorithm 6, computed by explicit
                            extraction of every window's feature vector
  * threshold            -- Section 4.4 (window is positive iff its distance
                            to the hyper-plane exceeds a given threshold)
  * NMS                  -- Section 3 (refinement by non-maximum suppression)

Readings of points the paper leaves open (each also listed in the design doc):
  R1 level k is resized from level 0 with pixel-centre-aligned bilinear
     interpolation in Q8 fixed point, rounded half up; level sizes are
     floor(W0 * den^k / num^k) for the scale num/den; levels are kept while
     the 64x128 window fits.
  R2 stencils clamp to the image edge (every pixel has a code / gradient).
  R3 LBP neighbour order TL,T,TR,R,BR,B,BL,L is bit 0..7; bit = 1 iff the
     neighbour is >= the centre (Section 4.2: lower gives 0, otherwise 1).
  R4 uniform LBP: codes with at most 2 circular 0/1 transitions (58 codes)
     take bins 0..57 in ascending code order; all others share bin 58.
  R5 gradient: dx = I[y][x-1] - I[y][x+1], dy = I[y-1][x] - I[y+1][x]
     (Algorithm 4), M = sqrt(dx^2 + dy^2), theta = atan2(dy, dx) in degrees
     folded to [0, 180).
  R6 9 orientation bins centred at 10 + 20k degrees, linear interpolation
     with wrap-around; spatial weights are bilinear to the two cell centres
     of the block in each axis; votes outside the block are dropped.
  R7 L2-Hys: v / sqrt(|v|^2 + eps^2), clip at 0.2, renormalise the same way,
     eps = 1e-3.
  R8 window (i, j) is anchored at cell (i, j) (stride 8 = one cell); its
     vector is the 15x7 HOG blocks then the 16x8 LBP cell histograms, both
     row-major with the channel innermost (3780 + 7552 = 11332 values).
  R9 threshold: over all windows of a frame, sort scores descending,
     k = ceil(0.01 N), t = (s_k + s_{k+1}) / 2; positive iff s > t.
  R10 greedy NMS on boxes in Q8 original-image pixels, order by score
     descending then (level, i, j) ascending, suppress iff IoU > 0.5
     (2 * inter > union in integers).
  R11 several models: window score = max over models, lowest model index on
     ties.
  R19 LBP block histograms (Algorithm 3): the raw sum of the 2x2 cell
     histograms of each 16x16 block (50 % overlap, no normalisation); a
     block-level window vector is the 15x7 HOG blocks then the 15x7 LBP
     blocks, row-major, channel innermost (3780 + 6195 = 9975 values).
"""
from __future__ import annotations

import math

import numpy as np

WIN_W, WIN_H = 64, 128          # window, Section 4.4
CELL = 8                        # 8x8 cells, Sections 4.2 and 4.3
HOG_BINS = 9
LBP_BINS = 59
WIN_BLOCKS_Y, WIN_BLOCKS_X = 15, 7   # HOG blocks per window
WIN_CELLS_Y, WIN_CELLS_X = 16, 8     # LBP cells per window
HOG_DIM = WIN_BLOCKS_Y * WIN_BLOCKS_X * 4 * HOG_BINS   # 3780
LBP_DIM = WIN_CELLS_Y * WIN_CELLS_X * LBP_BINS         # 7552
FEATURE_DIM = HOG_DIM + LBP_DIM                        # 11332
LBP_BLOCK_DIM = WIN_BLOCKS_Y * WIN_BLOCKS_X * LBP_BINS # 6195
BLOCK_MODEL_DIM = HOG_DIM + LBP_BLOCK_DIM              # 9975


# ---------------------------------------------------------------------------
# Pyramid (Section 4.4; Section 4.1 step 2; reading R1)
# ---------------------------------------------------------------------------

def level_sizes(w0: int, h0: int, scale_num: int = 11, scale_den: int = 10,
                max_levels: int = 0) -> list:
    """Exact level sizes (w_k, h_k) = floor(w0 den^k / num^k), kept while a
    64x128 window fits.  Integer arithmetic only."""
    sizes = []
    k = 0
    while True:
        wk = (w0 * scale_den ** k) // (scale_num ** k)
        hk = (h0 * scale_den ** k) // (scale_num ** k)
        if wk < WIN_W or hk < WIN_H:
            break
        sizes.append((wk, hk))
        k += 1
        if max_levels and k >= max_levels:
            break
    return sizes


def _axis_q8(n0: int, nk: int):
    """Q8 source coordinate of every output sample along one axis: the
    output sample centre (x + 0.5) maps to (x + 0.5) n0 / nk - 0.5 in the
    source; returns (index, fraction in 1/256, index + 1 clamped)."""
    x = np.arange(nk, dtype=np.int64)
    num = (2 * x + 1) * n0 - nk
    s = (num * 128) // nk
    i0 = s >> 8
    f = s & 255
    i1 = np.minimum(i0 + 1, n0 - 1)
    return i0, f, i1


def resize(img: np.ndarray, wk: int, hk: int) -> np.ndarray:
    """Level of size wk x hk from the uint8 level-0 image (reading R1)."""
    h0, w0 = img.shape
    x0, fx, x1 = _axis_q8(w0, wk)
    y0, fy, y1 = _axis_q8(h0, hk)
    p = img.astype(np.int64)
    fx = fx[None, :]
    fy = fy[:, None]
    p00 = p[y0][:, x0]
    p01 = p[y0][:, x1]
    p10 = p[y1][:, x0]
    p11 = p[y1][:, x1]
    acc = ((256 - fx) * (256 - fy) * p00 + fx * (256 - fy) * p01
           + (256 - fx) * fy * p10 + fx * fy * p11 + (1 << 15))
    return (acc >> 16).astype(np.uint8)


def pyramid(img: np.ndarray, scale_num: int = 11, scale_den: int = 10,
            max_levels: int = 0) -> list:
    h0, w0 = img.shape
    return [resize(img, wk, hk) for (wk, hk) in level_sizes(w0, h0, scale_num, scale_den, max_levels)]


# ---------------------------------------------------------------------------
# LBP (Section 4.2, Algorithms 1 and 2; readings R2-R4)
# ---------------------------------------------------------------------------

# (dy, dx) of neighbour k, k = 0..7: TL, T, TR, R, BR, B, BL, L
LBP_NEIGHBOURS = [(-1, -1), (-1, 0), (-1, 1), (0, 1), (1, 1), (1, 0), (1, -1), (0, -1)]


def lbp_codes(img: np.ndarray) -> np.ndarray:
    """8-bit LBP code of every pixel (Algorithm 1)."""
    h, w = img.shape
    p = np.pad(img.astype(np.int64), 1, mode="edge")
    c = p[1:h + 1, 1:w + 1]
    code = np.zeros((h, w), dtype=np.int64)
    for k, (dy, dx) in enumerate(LBP_NEIGHBOURS):
        n = p[1 + dy:1 + dy + h, 1 + dx:1 + dx + w]
        code += (n >= c).astype(np.int64) << k
    return code.astype(np.uint8)


def circular_transitions(code: int) -> int:
    bits = [(code >> k) & 1 for k in range(8)]
    return sum(bits[k] != bits[(k + 1) % 8] for k in range(8))


def uniform_bin_table() -> np.ndarray:
    """Map of the 256 codes to the 59 uniform-LBP bins (reading R4)."""
    table = np.full(256, LBP_BINS - 1, dtype=np.int64)
    nxt = 0
    for code in range(256):
        if circular_transitions(code) <= 2:
            table[code] = nxt
            nxt += 1
    assert nxt == LBP_BINS - 1
    return table


def lbp_cell_histograms(img: np.ndarray) -> np.ndarray:
    """Raw counts [Hc][Wc][59] of uniform-LBP bins per 8x8 cell
    (Algorithm 2).  Pixels beyond the last whole cell only act as
    neighbours."""
    h, w = img.shape
    hc, wc = h // CELL, w // CELL
    bins = uniform_bin_table()[lbp_codes(img).astype(np.int64)]
    hist = np.zeros((hc, wc, LBP_BINS), dtype=np.int64)
    for cy in range(hc):
        for cx in range(wc):
            cell = bins[cy * CELL:(cy + 1) * CELL, cx * CELL:(cx + 1) * CELL]
            hist[cy, cx] = np.bincount(cell.ravel(), minlength=LBP_BINS)
    return hist


# ---------------------------------------------------------------------------
# HOG (Section 4.3, Algorithms 4 and 5; readings R2, R5-R7)
# ---------------------------------------------------------------------------

def gradient(img: np.ndarray):
    """(dx, dy, magnitude, orientation in degrees in [0, 180)) per pixel,
    Algorithm 4 with edge clamping."""
    h, w = img.shape
    p = np.pad(img.astype(np.float64), 1, mode="edge")
    dx = p[1:h + 1, 0:w] - p[1:h + 1, 2:w + 2]
    dy = p[0:h, 1:w + 1] - p[2:h + 2, 1:w + 1]
    mag = np.sqrt(dx * dx + dy * dy)
    ang = np.degrees(np.arctan2(dy, dx))
    ang = np.where(ang < 0.0, ang + 180.0, ang)
    ang = np.where(ang >= 180.0, ang - 180.0, ang)
    return dx, dy, mag, ang


def orientation_votes(ang):
    """Two orientation bins and their weights for angles in [0, 180)
    (reading R6): bin centres at 10 + 20 k degrees, wrap-around."""
    t = np.asarray(ang, dtype=np.float64) / 20.0 - 0.5
    fl = np.floor(t)
    b0 = np.mod(fl, HOG_BINS).astype(np.int64)
    b1 = np.mod(b0 + 1, HOG_BINS)
    w1 = t - fl
    return b0, b1, 1.0 - w1, w1


def spatial_weight(p: int, slot: int) -> float:
    """Bilinear weight of pixel offset p in [0, 16) of a block towards the
    centre of the block's cell `slot` in {0, 1} along one axis."""
    u = (p + 0.5 - CELL / 2) / CELL
    return max(0.0, 1.0 - abs(u - slot))


def hog_block_histograms(mag: np.ndarray, ang: np.ndarray) -> np.ndarray:
    """Un-normalised block histograms [Hb][Wb][36], Algorithm 5: for every
    16x16 block (50 % overlap) every pixel of the block adds its magnitude
    into up to 2 cells x 2 cells x 2 orientation bins.  Slot layout
    (r * 2 + c) * 9 + bin."""
    h, w = mag.shape
    hb, wb = h // CELL - 1, w // CELL - 1
    if hb <= 0 or wb <= 0:
        return np.zeros((max(hb, 0), max(wb, 0), 4 * HOG_BINS))
    nblk = hb * wb
    flat = np.zeros(nblk * 4 * HOG_BINS)
    by = np.arange(hb)[:, None]
    bx = np.arange(wb)[None, :]
    block_index = (by * wb + bx)
    for py in range(2 * CELL):
        for px in range(2 * CELL):
            m = mag[CELL * by + py, CELL * bx + px]
            b0, b1, w0, w1 = orientation_votes(ang[CELL * by + py, CELL * bx + px])
            for r in (0, 1):
                wy = spatial_weight(py, r)
                if wy == 0.0:
                    continue
                for c in (0, 1):
                    wx = spatial_weight(px, c)
                    if wx == 0.0:
                        continue
                    base = (block_index * 4 + r * 2 + c) * HOG_BINS
                    flat += np.bincount((base + b0).ravel(), weights=(m * wy * wx * w0).ravel(),
                                        minlength=flat.size)
                    flat += np.bincount((base + b1).ravel(), weights=(m * wy * wx * w1).ravel(),
                                        minlength=flat.size)
    return flat.reshape(hb, wb, 4 * HOG_BINS)


def l2hys(v: np.ndarray, clip: float = 0.2, eps: float = 1e-3) -> np.ndarray:
    """L2-Hys over the last axis (reading R7)."""
    v = np.asarray(v, dtype=np.float64)
    v = v / np.sqrt(np.sum(v * v, axis=-1, keepdims=True) + eps * eps)
    v = np.minimum(v, clip)
    return v / np.sqrt(np.sum(v * v, axis=-1, keepdims=True) + eps * eps)


def hog_features(img: np.ndarray, clip: float = 0.2, eps: float = 1e-3) -> np.ndarray:
    """Normalised HOG block descriptors [Hb][Wb][36] of one level."""
    _, _, mag, ang = gradient(img)
    return l2hys(hog_block_histograms(mag, ang), clip, eps)


# ---------------------------------------------------------------------------
# Sliding window + linear SVM (Section 4.4, Algorithm 6; readings R8, R11)
# ---------------------------------------------------------------------------

def window_grid(wk: int, hk: int):
    """(rows, cols) of window anchors of a level: (Hc - 15, Wc - 7)."""
    hc, wc = hk // CELL, wk // CELL
    return max(0, hc - WIN_CELLS_Y + 1), max(0, wc - WIN_CELLS_X + 1)


def window_vector(hog: np.ndarray, cells: np.ndarray, i: int, j: int) -> np.ndarray:
    """Feature vector of the window anchored at cell (i, j)."""
    h = hog[i:i + WIN_BLOCKS_Y, j:j + WIN_BLOCKS_X, :]
    l = cells[i:i + WIN_CELLS_Y, j:j + WIN_CELLS_X, :]
    assert h.shape == (WIN_BLOCKS_Y, WIN_BLOCKS_X, 4 * HOG_BINS)
    assert l.shape == (WIN_CELLS_Y, WIN_CELLS_X, LBP_BINS)
    return np.concatenate([h.reshape(-1), l.reshape(-1).astype(np.float64)])


def window_scores(hog: np.ndarray, cells: np.ndarray, weights: np.ndarray,
                  bias: np.ndarray, chunk: int = 512) -> np.ndarray:
    """Scores [m][Y][X] = <x_window, w_m> + b_m by explicit extraction of
    every window vector (brute force)."""
    weights = np.atleast_2d(np.asarray(weights, dtype=np.float64))
    bias = np.asarray(bias, dtype=np.float64).reshape(-1)
    m = weights.shape[0]
    ny = max(0, cells.shape[0] - WIN_CELLS_Y + 1)
    nx = max(0, cells.shape[1] - WIN_CELLS_X + 1)
    out = np.zeros((m, ny, nx))
    anchors = [(i, j) for i in range(ny) for j in range(nx)]
    for s in range(0, len(anchors), chunk):
        part = anchors[s:s + chunk]
        x = np.stack([window_vector(hog, cells, i, j) for (i, j) in part])
        sc = x @ weights.T + bias[None, :]
        for q, (i, j) in enumerate(part):
            out[:, i, j] = sc[q]
    return out


def level_features(level: np.ndarray, clip: float = 0.2, eps: float = 1e-3):
    return hog_features(level, clip, eps), lbp_cell_histograms(level)


# ---------------------------------------------------------------------------
# LBP block histograms (Section 4.2, Algorithm 3; reading R19) and the
# cell-level model with the same scores
# ---------------------------------------------------------------------------

def lbp_block_histograms(cells: np.ndarray) -> np.ndarray:
    """[Hb][Wb][59]: each 16x16 block's histogram is the sum of its four
    8x8 cell histograms (the histogram reduction of Algorithm 3)."""
    cells = np.asarray(cells, dtype=np.int64)
    return cells[:-1, :-1] + cells[:-1, 1:] + cells[1:, :-1] + cells[1:, 1:]


def window_vector_blocks(hog: np.ndarray, lbp_blocks: np.ndarray, i: int, j: int) -> np.ndarray:
    """Block-level feature vector of the window anchored at cell (i, j)."""
    h = hog[i:i + WIN_BLOCKS_Y, j:j + WIN_BLOCKS_X, :]
    l = lbp_blocks[i:i + WIN_BLOCKS_Y, j:j + WIN_BLOCKS_X, :]
    assert h.shape == (WIN_BLOCKS_Y, WIN_BLOCKS_X, 4 * HOG_BINS)
    assert l.shape == (WIN_BLOCKS_Y, WIN_BLOCKS_X, LBP_BINS)
    return np.concatenate([h.reshape(-1), l.reshape(-1).astype(np.float64)])


def window_scores_blocks(hog: np.ndarray, lbp_blocks: np.ndarray, weights: np.ndarray,
                         bias: np.ndarray) -> np.ndarray:
    """Scores [m][Y][X] of block-level models [m][9975] by explicit
    extraction of every window's block-level vector (brute force)."""
    weights = np.atleast_2d(np.asarray(weights, dtype=np.float64))
    bias = np.asarray(bias, dtype=np.float64).reshape(-1)
    ny = max(0, lbp_blocks.shape[0] - WIN_BLOCKS_Y + 1)
    nx = max(0, lbp_blocks.shape[1] - WIN_BLOCKS_X + 1)
    out = np.zeros((weights.shape[0], ny, nx))
    for i in range(ny):
        x = np.stack([window_vector_blocks(hog, lbp_blocks, i, j) for j in range(nx)]) if nx else None
        if nx:
            out[:, i, :] = (x @ weights.T + bias[None, :]).T
    return out


def fold_lbp_block_weights(weights: np.ndarray) -> np.ndarray:
    """The cell-level model [m][11332] that scores every window as the
    block-level model [m][9975] does: HOG weights copied; since a block
    histogram is the plain sum of its cells, the weight of window cell
    (a, b) is the sum of the weights of the window blocks that contain it,
    (a', b') with a' in {a-1, a} and b' in {b-1, b}."""
    weights = np.atleast_2d(np.asarray(weights, dtype=np.float64))
    m = weights.shape[0]
    out = np.zeros((m, FEATURE_DIM))
    out[:, :HOG_DIM] = weights[:, :HOG_DIM]
    wb = weights[:, HOG_DIM:].reshape(m, WIN_BLOCKS_Y, WIN_BLOCKS_X, LBP_BINS)
    wc = np.zeros((m, WIN_CELLS_Y, WIN_CELLS_X, LBP_BINS))
    for a in range(WIN_CELLS_Y):
        for b in range(WIN_CELLS_X):
            for a2 in (a - 1, a):
                for b2 in (b - 1, b):
                    if 0 <= a2 < WIN_BLOCKS_Y and 0 <= b2 < WIN_BLOCKS_X:
                        wc[:, a, b, :] += wb[:, a2, b2, :]
    out[:, HOG_DIM:] = wc.reshape(m, -1)
    return out


# ---------------------------------------------------------------------------
# Threshold, boxes, NMS (Section 4.4 classification; Section 3 refinement;
# readings R9-R11)
# ---------------------------------------------------------------------------

def threshold_99(scores) -> float:
    """Midpoint between the k-th and (k+1)-th largest score, k = ceil(N/100)."""
    s = np.sort(np.asarray(scores, dtype=np.float64).ravel())[::-1]
    n = s.size
    if n == 0:
        return math.inf
    k = math.ceil(0.01 * n)
    if k >= n:
        return -math.inf
    return 0.5 * (s[k - 1] + s[k])


def window_box_q8(w0: int, h0: int, wk: int, hk: int, i: int, j: int):
    """Window (i, j) of a level of size wk x hk as an integer box in 1/256
    pixels of the original w0 x h0 image: (x0, y0, x1, y1)."""
    x0 = (256 * CELL * j * w0) // wk
    x1 = (256 * (CELL * j + WIN_W) * w0) // wk
    y0 = (256 * CELL * i * h0) // hk
    y1 = (256 * (CELL * i + WIN_H) * h0) // hk
    return x0, y0, x1, y1


def iou_exceeds_half(a, b) -> bool:
    """IoU(a, b) > 0.5 decided exactly in integers: 2 inter > union."""
    iw = min(a[2], b[2]) - max(a[0], b[0])
    ih = min(a[3], b[3]) - max(a[1], b[1])
    if iw <= 0 or ih <= 0:
        return False
    inter = iw * ih
    union = (a[2] - a[0]) * (a[3] - a[1]) + (b[2] - b[0]) * (b[3] - b[1]) - inter
    return 2 * inter > union


def nms(cands: list) -> list:
    """Greedy non-maximum suppression.  `cands` holds dicts with keys
    score, level, i, j, box; returns the kept ones in processing order."""
    order = sorted(cands, key=lambda c: (-c["score"], c["level"], c["i"], c["j"]))
    removed = [False] * len(order)
    kept = []
    for a in range(len(order)):
        if removed[a]:
            continue
        kept.append(order[a])
        for b in range(a + 1, len(order)):
            if not removed[b] and iou_exceeds_half(order[a]["box"], order[b]["box"]):
                removed[b] = True
    return kept


def select_top(cands: list, limit: int) -> list:
    """The `limit` first candidates in the NMS order (score descending, then
    level, i, j ascending): the ones NMS takes when a frame has more than it
    holds (the candidate list is not refined past that many; a reading, the
    paper fixes no such limit)."""
    return sorted(cands, key=lambda c: (-c["score"], c["level"], c["i"], c["j"]))[:limit]


def max_over_models(scores: np.ndarray):
    """(max score, argmax model with lowest index on ties) over axis 0."""
    scores = np.asarray(scores, dtype=np.float64)
    return scores.max(axis=0), scores.argmax(axis=0)


# ---------------------------------------------------------------------------
# Whole frame
# ---------------------------------------------------------------------------

def frame_scores(img: np.ndarray, weights: np.ndarray, bias: np.ndarray,
                 scale_num: int = 11, scale_den: int = 10, max_levels: int = 0,
                 clip: float = 0.2, eps: float = 1e-3) -> list:
    """Per level: dict(size, level image, hog, cells, scores [m][Y][X])."""
    out = []
    for lv in pyramid(img, scale_num, scale_den, max_levels):
        hog, cells = level_features(lv, clip, eps)
        sc = window_scores(hog, cells, weights, bias)
        out.append({"size": (lv.shape[1], lv.shape[0]), "image": lv, "hog": hog,
                    "cells": cells, "scores": sc})
    return out


def frame_threshold(levels: list) -> float:
    allmax = [max_over_models(lv["scores"])[0].ravel() for lv in levels]
    return threshold_99(np.concatenate(allmax) if allmax else np.zeros(0))


def candidates(levels: list, w0: int, h0: int, thr: float) -> list:
    """Windows whose (max-over-models) score exceeds the threshold."""
    out = []
    for k, lv in enumerate(levels):
        wk, hk = lv["size"]
        s, m = max_over_models(lv["scores"])
        for i, j in zip(*np.nonzero(s > thr)):
            out.append({"score": float(s[i, j]), "level": k, "i": int(i), "j": int(j),
                        "model": int(m[i, j]), "box": window_box_q8(w0, h0, wk, hk, int(i), int(j))})
    return out


def detect(img: np.ndarray, weights: np.ndarray, bias: np.ndarray, thr: float = None,
           scale_num: int = 11, scale_den: int = 10, max_levels: int = 0):
    """Full pipeline: returns (levels, threshold, candidates, kept)."""
    h0, w0 = img.shape
    levels = frame_scores(img, weights, bias, scale_num, scale_den, max_levels)
    if thr is None:
        thr = frame_threshold(levels)
    cands = candidates(levels, w0, h0, thr)
    return levels, thr, cands, nms(cands)
