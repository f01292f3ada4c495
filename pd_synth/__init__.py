"""Seeded synthetic inputs for the pedestrian-detection hot path.

Both the HIP path (tests, bench) and the CPU oracle draw their inputs from
here.  This module holds none of the detection method's arithmetic: it only
makes frames that look like the paper's workload (8-bit grayscale road
frames of 1242x375, Section 5.1) and seeded linear-SVM weight vectors (the
paper's SVM is trained offline on data that is not available, Section 4.4).

Frame recipe (frame f uses seed 1000 + f unless a seed is given):
  * background: a coarse grid at 1/16 resolution, uniform in [48, 208],
    upsampled with separable linear interpolation, plus N(0, 4^2) noise;
  * 20 objects: 75 % filled rectangles (width U[8, W/4], height
    U[16, H/2], bright U[200, 255] or dark U[0, 55], 50/50), 25 % straight
    step edges (a random line through the frame; one side is offset by
    +-U[30, 80]);
  * clip to [0, 255], round half to even, uint8.
SVM weights: model m uses seed 7 + m, w ~ N(0, 0.01^2) rounded to float32,
bias 0.
"""
from __future__ import annotations

import numpy as np

FEATURE_DIM = 3780 + 7552  # HOG 15x7 blocks x 36 + LBP 16x8 cells x 59

__all__ = [
    "FEATURE_DIM",
    "frame",
    "frame_batch",
    "svm_weights",
    "svm_bias",
    "CONFIG_SIZES",
]

# Frame sizes of the named workloads: (width, height) per frame.
CONFIG_SIZES = {
    "small": [(320, 240)],
    "road": [(1242, 375)],
    "mixed64": [(640, 480)] * 24 + [(1242, 375)] * 24 + [(1920, 1080)] * 16,
    "road16": [(1242, 375)] * 16,
}


def _upsample_linear(grid: np.ndarray, height: int, width: int, step: int) -> np.ndarray:
    gh, gw = grid.shape
    ys = (np.arange(height) + 0.5) / step - 0.5
    xs = (np.arange(width) + 0.5) / step - 0.5
    ys = np.clip(ys, 0, gh - 1)
    xs = np.clip(xs, 0, gw - 1)
    y0 = np.minimum(np.floor(ys).astype(np.int64), gh - 2)
    x0 = np.minimum(np.floor(xs).astype(np.int64), gw - 2)
    ty = (ys - y0)[:, None]
    tx = (xs - x0)[None, :]
    g00 = grid[y0][:, x0]
    g01 = grid[y0][:, x0 + 1]
    g10 = grid[y0 + 1][:, x0]
    g11 = grid[y0 + 1][:, x0 + 1]
    top = g00 * (1 - tx) + g01 * tx
    bot = g10 * (1 - tx) + g11 * tx
    return top * (1 - ty) + bot * ty


def frame(width: int, height: int, seed: int, n_objects: int = 20) -> np.ndarray:
    """One synthetic uint8 grayscale frame of shape [height][width]."""
    if width <= 0 or height <= 0:
        return np.zeros((max(height, 0), max(width, 0)), dtype=np.uint8)
    rng = np.random.default_rng(seed)
    step = 16
    gh = max(2, -(-height // step) + 2)
    gw = max(2, -(-width // step) + 2)
    grid = rng.uniform(48.0, 208.0, size=(gh, gw))
    img = _upsample_linear(grid, height, width, step)
    img = img + rng.normal(0.0, 4.0, size=(height, width))
    yy, xx = np.mgrid[0:height, 0:width]
    for _ in range(n_objects):
        if rng.random() < 0.75:
            w = int(rng.integers(8, max(9, width // 4 + 1)))
            h = int(rng.integers(16, max(17, height // 2 + 1)))
            x0 = int(rng.integers(-w // 2, width))
            y0 = int(rng.integers(-h // 2, height))
            if rng.random() < 0.5:
                val = rng.uniform(200.0, 255.0)
            else:
                val = rng.uniform(0.0, 55.0)
            ys, ye = max(0, y0), min(height, y0 + h)
            xs, xe = max(0, x0), min(width, x0 + w)
            if ys < ye and xs < xe:
                img[ys:ye, xs:xe] = val + rng.normal(0.0, 4.0, size=(ye - ys, xe - xs))
        else:
            px = rng.uniform(0, width)
            py = rng.uniform(0, height)
            ang = rng.uniform(0.0, np.pi)
            off = rng.uniform(30.0, 80.0) * (1 if rng.random() < 0.5 else -1)
            side = (xx - px) * np.sin(ang) - (yy - py) * np.cos(ang) > 0
            img = img + off * side
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def frame_batch(sizes, seed0: int = 1000) -> list:
    """Frames for a list of (width, height); frame f uses seed seed0 + f."""
    return [frame(w, h, seed0 + f) for f, (w, h) in enumerate(sizes)]


def svm_weights(n_models: int = 1, dim: int = FEATURE_DIM, seed0: int = 7) -> np.ndarray:
    """Seeded linear-SVM weights, float32 [n_models][dim]; model m uses seed seed0 + m."""
    out = np.empty((n_models, dim), dtype=np.float32)
    for m in range(n_models):
        out[m] = np.random.default_rng(seed0 + m).normal(0.0, 0.01, size=dim).astype(np.float32)
    return out


def svm_bias(n_models: int = 1) -> np.ndarray:
    return np.zeros(n_models, dtype=np.float32)


PRUNER_CHANNELS = (68, 32, 32, 16)


def pruner_init(channels=PRUNER_CHANNELS, seed: int = 11) -> np.ndarray:
    """Initial parameters of the window pruner as one float32 vector, laid out
    per conv layer as weights [Cout][Cin][3][3] then bias [Cout], then the 1x1
    head's weights [C] and bias: He-normal weights (std sqrt(2 / (9 Cin)),
    head std sqrt(1 / C)), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (9 * cin)), cout * cin * 9))
        parts.append(np.zeros(cout))
    parts.append(rng.normal(0.0, np.sqrt(1.0 / channels[-1]), channels[-1]))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)
