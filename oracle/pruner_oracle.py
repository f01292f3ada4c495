"""Plain FP64 CPU oracle for the learned window pruner.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares no code with
the HIP path; both sides draw their inputs (frames, initial network weights)
from the seeded generator package `pd_synth`.

The pruner is not part of the paper.  It is a small convolutional network
that looks at a per-cell feature map built from the paper's own cell-level
quantities and predicts, for every sliding window, whether the linear SVM of
Section 4.4 will score it above the threshold; windows it rejects are not
scored.  Everything below is the definition of each quantity, written for
readability:

  * cell map (68 channels per 8x8 cell):
      - 9 HOG channels: the cell's orientation histogram (Section 4.3 gradient
        and orientation binning, Algorithm 4 and the linear orientation vote
        of Algorithm 5) with the full bilinear spatial kernel -- every pixel
        whose centre lies within 8 pixels (per axis) of the cell centre votes
        with weight (1 - |dy|/8)(1 - |dx|/8); pixels outside the cell grid do
        not vote -- then divided by sqrt(|h|^2 + eps^2), eps = 1e-3;
      - 59 LBP channels: the uniform-LBP cell histogram (Section 4.2,
        Algorithms 1-2) divided by 64.
  * network: conv3x3 68->32, ReLU, conv3x3 32->32, ReLU, conv3x3 32->16,
    ReLU, 1x1 16->1, sigmoid; zero "same" padding; one logit per cell.
  * window (i, j) takes the logit of cell (i + 7, j + 3).
  * training loss: binary cross-entropy over the cells that carry a window,
    positives weighted by pos_weight, mean over those cells.
  * Adam (Kingma and Ba) with bias correction.
  * pruning: per frame, keep the windows whose logit is >= the K-th largest
    logit among the frame's windows; a window is a candidate iff it is kept
    and its SVM score exceeds the threshold.
  * recall: plain post-NMS detections matched one to one by pruned post-NMS
    detections with IoU >= 0.5 (greedy, plain detections in NMS order, each
    taking the unmatched pruned box of largest IoU, earliest on ties).

Parameter vector layout (float, 33,505 values for 68/32/32/16):
  for each conv layer l: weights [Cout][Cin][3][3], then bias [Cout];
  then the head: weights [16], bias [1].
"""
from __future__ import annotations

import numpy as np

from . import pd_oracle as O

CHANNELS = (68, 32, 32, 16)      # cell-map channels, then conv outputs
HOG_CH, LBP_CH = 9, 59
WIN_CELL_OFFSET = (7, 3)          # window (i, j) <-> cell (i + 7, j + 3)


# ---------------------------------------------------------------- cell map --
def cell_hog_full(img: np.ndarray) -> np.ndarray:
    """Un-normalised 9-bin cell histograms [Hc][Wc][9] with the full bilinear
    spatial kernel: for every target cell, every pixel of the cell grid within
    the 16x16 square centred on the cell centre votes mag * (orientation
    weight) * (1 - |y + 0.5 - yc| / 8) * (1 - |x + 0.5 - xc| / 8)."""
    h, w = img.shape
    hc, wc = h // O.CELL, w // O.CELL
    out = np.zeros((hc, wc, HOG_CH))
    if hc == 0 or wc == 0:
        return out
    _, _, mag, ang = O.gradient(img)
    b0, b1, w0, w1 = O.orientation_votes(ang)
    gh, gw = O.CELL * hc, O.CELL * wc           # pixels inside the cell grid
    for ty in range(hc):
        yc = O.CELL * ty + O.CELL / 2
        ys = np.arange(max(0, int(yc) - O.CELL), min(gh, int(yc) + O.CELL))
        wy = 1.0 - np.abs(ys + 0.5 - yc) / O.CELL
        for tx in range(wc):
            xc = O.CELL * tx + O.CELL / 2
            xs = np.arange(max(0, int(xc) - O.CELL), min(gw, int(xc) + O.CELL))
            wx = 1.0 - np.abs(xs + 0.5 - xc) / O.CELL
            sp = wy[:, None] * wx[None, :]
            m = mag[np.ix_(ys, xs)] * sp
            hist = np.bincount(b0[np.ix_(ys, xs)].ravel(), weights=(m * w0[np.ix_(ys, xs)]).ravel(),
                               minlength=HOG_CH)
            hist += np.bincount(b1[np.ix_(ys, xs)].ravel(), weights=(m * w1[np.ix_(ys, xs)]).ravel(),
                                minlength=HOG_CH)
            out[ty, tx] = hist
    return out


def cellmap(img: np.ndarray, eps: float = 1e-3) -> np.ndarray:
    """Cell map [Hc][Wc][68] of one pyramid level: 9 normalised HOG channels,
    then 59 LBP counts / 64."""
    hog = cell_hog_full(img)
    hog = hog / np.sqrt(np.sum(hog * hog, axis=-1, keepdims=True) + eps * eps)
    lbp = O.lbp_cell_histograms(img).astype(np.float64) / 64.0
    return np.concatenate([hog, lbp], axis=-1)


# ----------------------------------------------------------------- network --
def param_count(ch=CHANNELS) -> int:
    n = 0
    for cin, cout in zip(ch[:-1], ch[1:]):
        n += cout * cin * 9 + cout
    return n + ch[-1] + 1


def unpack(params: np.ndarray, ch=CHANNELS):
    """[(W [Cout][Cin][3][3], b [Cout]) per conv layer], (head w [C], head b)."""
    p = np.asarray(params, dtype=np.float64)
    layers, o = [], 0
    for cin, cout in zip(ch[:-1], ch[1:]):
        wgt = p[o:o + cout * cin * 9].reshape(cout, cin, 3, 3)
        o += cout * cin * 9
        layers.append((wgt, p[o:o + cout]))
        o += cout
    hw = p[o:o + ch[-1]]
    hb = p[o + ch[-1]]
    assert o + ch[-1] + 1 == p.size
    return layers, (hw, hb)


def pack(layers, head) -> np.ndarray:
    parts = []
    for wgt, b in layers:
        parts += [np.ravel(wgt), np.ravel(b)]
    parts += [np.ravel(head[0]), np.atleast_1d(head[1])]
    return np.concatenate(parts).astype(np.float64)


def conv3x3(x: np.ndarray, wgt: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[p][q][o] = b[o] + sum_{c, u, v} W[o][c][u][v] x[p + u - 1][q + v - 1][c],
    zero outside the map.  x: [H][W][Cin]."""
    h, w, cin = x.shape
    xp = np.zeros((h + 2, w + 2, cin))
    xp[1:h + 1, 1:w + 1] = x
    y = np.zeros((h, w, wgt.shape[0])) + b
    for u in range(3):
        for v in range(3):
            y += xp[u:u + h, v:v + w] @ wgt[:, :, u, v].T
    return y


def forward(x: np.ndarray, params: np.ndarray, ch=CHANNELS):
    """(logits [H][W], cache of every layer's input and pre-activation)."""
    layers, (hw, hb) = unpack(params, ch)
    cache = []
    a = x
    for wgt, b in layers:
        z = conv3x3(a, wgt, b)
        cache.append((a, z))
        a = np.maximum(z, 0.0)
    logit = a @ hw + hb
    cache.append((a, None))
    return logit, cache


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def bce_loss_grad(logits_list, labels_list, masks_list, pos_weight: float):
    """(loss, [dL/dlogit per map]) for the masked binary cross-entropy with
    positives weighted by pos_weight, averaged over every masked cell of the
    batch."""
    n = sum(float(m.sum()) for m in masks_list)
    loss, grads = 0.0, []
    for z, y, m in zip(logits_list, labels_list, masks_list):
        z = np.asarray(z, dtype=np.float64)
        s = sigmoid(z)
        # log(sigmoid(z)) and log(1 - sigmoid(z)) written stably
        log_s = -np.logaddexp(0.0, -z)
        log_1ms = -np.logaddexp(0.0, z)
        loss += float(np.sum(m * (-pos_weight * y * log_s - (1.0 - y) * log_1ms)))
        grads.append(m * ((1.0 - y) * s - pos_weight * y * (1.0 - s)) / n)
    return loss / n, grads


def backward(dlogit: np.ndarray, cache, params: np.ndarray, ch=CHANNELS) -> np.ndarray:
    """Gradient of the parameters (packed like `params`) for one map, given
    dL/dlogit [H][W] and the forward cache."""
    layers, (hw, hb) = unpack(params, ch)
    a3, _ = cache[-1]
    g_hw = np.einsum("pq,pqc->c", dlogit, a3)
    g_hb = float(dlogit.sum())
    da = dlogit[:, :, None] * hw[None, None, :]
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        wgt, _ = layers[li]
        a_in, z = cache[li]
        dz = da * (z > 0.0)
        h, w, cin = a_in.shape
        xp = np.zeros((h + 2, w + 2, cin))
        xp[1:h + 1, 1:w + 1] = a_in
        gw = np.zeros_like(wgt)
        dxp = np.zeros((h + 2, w + 2, cin))
        for u in range(3):
            for v in range(3):
                patch = xp[u:u + h, v:v + w]
                gw[:, :, u, v] = np.einsum("pqo,pqc->oc", dz, patch)
                dxp[u:u + h, v:v + w] += dz @ wgt[:, :, u, v]
        grads.append((gw, dz.sum(axis=(0, 1))))
        da = dxp[1:h + 1, 1:w + 1]
    grads.reverse()
    return pack(grads, (g_hw, g_hb))


def adam_step(params, grad, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ----------------------------------------------------- labels and pruning --
def window_labels(hc: int, wc: int, scores: np.ndarray, thr: float):
    """(labels, mask) [Hc][Wc] of one level: the cell of window (i, j) is
    labelled 1 iff the window's score (max over models) exceeds thr; cells
    that carry no window are masked out."""
    lab = np.zeros((hc, wc))
    mask = np.zeros((hc, wc))
    ny, nx = scores.shape
    di, dj = WIN_CELL_OFFSET
    mask[di:di + ny, dj:dj + nx] = 1.0
    lab[di:di + ny, dj:dj + nx] = (scores > thr).astype(np.float64)
    return lab, mask


def window_logits(logit_map: np.ndarray, ny: int, nx: int) -> np.ndarray:
    di, dj = WIN_CELL_OFFSET
    return logit_map[di:di + ny, dj:dj + nx]


def keep_topk(window_logit_levels, k: int):
    """Per frame: boolean keep masks per level, keeping every window whose
    logit is >= the k-th largest of the frame (ties kept)."""
    allz = np.concatenate([z.ravel() for z in window_logit_levels])
    if k <= 0 or allz.size == 0:
        return [np.zeros(z.shape, bool) for z in window_logit_levels]
    kth = np.sort(allz)[::-1][min(k, allz.size) - 1]
    return [z >= kth for z in window_logit_levels]


def match_recall(plain_boxes, pruned_boxes) -> float:
    """Fraction of plain detections matched one to one (IoU >= 0.5) by pruned
    detections; boxes are (x0, y0, x1, y1) integer tuples, plain ones in NMS
    order."""
    if not plain_boxes:
        return 1.0
    used = [False] * len(pruned_boxes)
    hit = 0
    for a in plain_boxes:
        best, best_iou = -1, -1.0
        for q, b in enumerate(pruned_boxes):
            if used[q]:
                continue
            iw = min(a[2], b[2]) - max(a[0], b[0])
            ih = min(a[3], b[3]) - max(a[1], b[1])
            inter = max(iw, 0) * max(ih, 0)
            union = (a[2] - a[0]) * (a[3] - a[1]) + (b[2] - b[0]) * (b[3] - b[1]) - inter
            if 2 * inter >= union and union > 0:
                iou = inter / union
                if iou > best_iou:
                    best, best_iou = q, iou
        if best >= 0:
            used[best] = True
            hit += 1
    return hit / len(plain_boxes)
