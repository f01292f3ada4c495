"""Training and calibration of the learned window pruner, on the GPU.

Orchestration only: every array operation below is one of libpd's kernels
(cell maps, scores, labels, forward, backward, Adam, detection).  Torch
provides device memory and a few scalar reductions for bookkeeping.

* training set: for each frame, every pyramid level's cell map
  (pd_features_cellmap) and labels from the plain detector's window scores
  (max over models) against the detection threshold (pd_window_labels);
* training: class-weighted BCE (positive weight = negatives / positives over
  the training set), Adam with FP32 master weights, a fixed number of frames
  per step, steps in a seeded random order per epoch (epoch e's order depends
  on (seed, e) only); a checkpoint (parameters, Adam moments, step, seed) can
  be written after every epoch and training resumed from it bitwise;
* calibration: the smallest per-frame K at which the pruned detector's
  post-NMS boxes recall at least the target fraction of the plain detector's
  (one-to-one matching at IoU >= 0.5, greedy in the plain NMS order) over a
  held-out set.
"""
from __future__ import annotations

import numpy as np

from . import (Detector, PrunerBatch, adam_step, build_pyramid, features_cellmap, params as make_params,
               pruner_load, pruner_save, score_windows, window_labels, PRUNER_PARAMS)


def _torch():
    import torch
    return torch


def level_maps(frame, weights, bias, threshold_dev, prm):
    """[(cell map, labels, mask)] of every level of one device frame."""
    _, _, views = build_pyramid(frame, prm)
    out = []
    for v in views:
        blocks, cells, cmap = features_cellmap(v.contiguous(), prm)
        s = score_windows(blocks, cells, weights, bias).max(dim=0).values
        lab, mask = window_labels(s, int(cmap.shape[2]), int(cmap.shape[1]), threshold_dev)
        out.append((cmap, lab, mask))
    return out


def training_set(frames, weights, bias, threshold, prm=None):
    """Per frame, the list of its levels' (cell map, labels, mask); threshold:
    one value for every frame, or a sequence of one per frame."""
    torch = _torch()
    prm = prm or make_params()
    thr = list(threshold) if hasattr(threshold, "__len__") else [threshold] * len(frames)
    return [level_maps(f, weights, bias, torch.tensor([t], dtype=torch.float64, device=frames[0].device), prm)
            for f, t in zip(frames, thr)]


def train(data, init_params, epochs: int = 4, frames_per_step: int = 8, lr: float = 1e-3, seed: int = 0,
          log=None, checkpoint: str = None, resume: str = None):
    """Trains from `init_params` (device float32 [PRUNER_PARAMS]) for
    `epochs` epochs; returns (params, per-epoch mean loss list, positive
    weight).  checkpoint: a file written (pd_pruner_save) after every epoch.
    resume: a checkpoint of this training (same data, steps per epoch and
    learning rate) to continue from: its parameters, moments, step and seed
    replace init_params and `seed`, and only the epochs after it run (the
    returned losses are theirs)."""
    torch = _torch()
    dev = init_params.device
    n_pos = sum(float(lab.sum()) for frame in data for _, lab, _ in frame)
    n_all = sum(float(mask.sum()) for frame in data for _, _, mask in frame)
    pos_weight = (n_all - n_pos) / max(n_pos, 1.0)
    p = init_params.clone().contiguous()
    assert p.numel() == PRUNER_PARAMS
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    t = 0
    if resume is not None:
        t, seed = pruner_load(resume, p, m, v)
    steps = [data[i:i + frames_per_step] for i in range(0, len(data), frames_per_step)]
    batches, ws = [], None
    for group in steps:
        maps = [lv for frame in group for lv in frame]
        b = PrunerBatch([c for c, _, _ in maps], [l for _, l, _ in maps], [k for _, _, k in maps], workspace=ws)
        ws = b.workspace if ws is None or b.workspace.numel() > ws.numel() else ws
        batches.append(b)
    if t % len(batches):
        raise ValueError(f"checkpoint step {t} is not a whole number of {len(batches)}-step epochs")
    history = []
    for ep in range(t // len(batches), epochs):
        loss = torch.zeros((), dtype=torch.float64, device=dev)
        for k in np.random.default_rng([seed, ep]).permutation(len(batches)):
            b = batches[k]
            b.gradient(p, pos_weight)
            t += 1
            adam_step(p, b.grad, m, v, t, lr=lr)
            loss += b.stats[0]
        history.append(float(loss) / len(batches))
        if checkpoint is not None:
            pruner_save(checkpoint, p, m, v, t, seed)
        if log:
            log(f"epoch {ep}: mean loss {history[-1]:.4f}")
    return p, history, pos_weight


def match_recall(plain, pruned) -> float:
    """Fraction of `plain` boxes (structured pd_box rows in NMS order)
    matched one to one by `pruned` boxes with IoU >= 0.5 (2 inter >= union),
    each plain box taking the unmatched pruned box of largest IoU."""
    if len(plain) == 0:
        return 1.0
    pb = np.stack([pruned[q].astype(np.int64) for q in ("x0", "y0", "x1", "y1")], axis=1) if len(pruned) else \
        np.zeros((0, 4), np.int64)
    used = np.zeros(len(pb), bool)
    hit = 0
    for row in plain:
        a = [int(row[q]) for q in ("x0", "y0", "x1", "y1")]
        iw = np.minimum(a[2], pb[:, 2]) - np.maximum(a[0], pb[:, 0])
        ih = np.minimum(a[3], pb[:, 3]) - np.maximum(a[1], pb[:, 1])
        inter = np.maximum(iw, 0) * np.maximum(ih, 0)
        union = (a[2] - a[0]) * (a[3] - a[1]) + (pb[:, 2] - pb[:, 0]) * (pb[:, 3] - pb[:, 1]) - inter
        ok = (2 * inter >= union) & (union > 0) & ~used
        if ok.any():
            iou = np.where(ok, inter / np.maximum(union, 1), -1.0)
            q = int(np.argmax(iou))
            used[q] = True
            hit += 1
    return hit / len(plain)


def recall_at(frames, weights, bias, thresholds, pruner, keep: int, plain_boxes, prm_kw=None):
    """(recall over all frames' plain boxes, pruned boxes) at per-frame K = keep."""
    prm_kw = dict(prm_kw or {})
    det = Detector(frames, weights, bias, make_params(prune_keep=keep, pruner=pruner, **prm_kw), cap=1024)
    det.run(thresholds)
    _torch().cuda.synchronize()
    boxes, counts = det.results()
    total = sum(len(b) for b in plain_boxes)
    hit = sum(match_recall(a, b) * len(a) for a, b in zip(plain_boxes, boxes))
    return (hit / total if total else 1.0), boxes


def calibrate_keep(frames, weights, bias, thresholds, pruner, target: float = 0.99, prm_kw=None, plain_kw=None):
    """Smallest K (binary search over [1, windows per frame]) whose recall
    over `frames` reaches `target`; returns (K, recall, plain boxes, windows
    per frame).  prm_kw: params of the pruned detector; plain_kw: of the
    plain detector it is measured against (default: the same)."""
    prm_kw = dict(prm_kw or {})
    plain_kw = dict(prm_kw if plain_kw is None else plain_kw)
    det = Detector(frames, weights, bias, make_params(**plain_kw), cap=1024)
    det.run(thresholds)
    _torch().cuda.synchronize()
    plain, _ = det.results()
    n_win = max(windows_per_frame(int(f.shape[1]), int(f.shape[0]), make_params(**prm_kw)) for f in frames)
    lo, hi = 1, max(n_win, 1)
    best = (hi, 1.0)
    while lo < hi:
        mid = (lo + hi) // 2
        r, _ = recall_at(frames, weights, bias, thresholds, pruner, mid, plain, prm_kw)
        if r >= target:
            hi = mid
            best = (mid, r)
        else:
            lo = mid + 1
    if best[0] != lo:
        best = (lo, recall_at(frames, weights, bias, thresholds, pruner, lo, plain, prm_kw)[0])
    return best[0], best[1], plain, n_win


def windows_per_frame(w: int, h: int, prm=None) -> int:
    from . import plan_pyramid
    levels, _ = plan_pyramid(w, h, prm or make_params())
    return sum(L.win_x * L.win_y for L in levels)
