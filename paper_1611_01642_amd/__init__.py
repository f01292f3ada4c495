"""Python binding of libpd, the MI355X HOG+LBP+SVM detection hot path.

Argument marshalling only: every step runs in libpd's HIP kernels.  Torch
tensors serve as device memory (``data_ptr()``) and streams
(``torch.cuda.current_stream()``).  If libpd.so has not been built this module
raises on first use; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpd.so")

CELL = 8
WIN_W, WIN_H = 64, 128
HOG_BLOCK = 36
LBP_BINS = 59
HOG_DIM, LBP_DIM, FEATURE_DIM = 3780, 7552, 11332
LBP_BLOCK_DIM, BLOCK_MODEL_DIM = 6195, 9975
MAX_LEVELS = 64
MAX_MODELS = 16
MAX_CANDIDATES = 4096
FEAT_HOG, FEAT_LBP = 1, 2
PREC_F32, PREC_BF16 = 0, 1
MAX_MODELS_BF16 = 8
PRUNER_CHANNELS, PRUNER_PARAMS = 68, 33505
NOALLOC_SCRATCH_BYTES = 64 << 20

E_ARG, E_SIZE, E_WORKSPACE, E_HIP, E_OVERFLOW, E_IO = -1, -2, -3, -4, -5, -6


class PdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libpd error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("scale_num", ctypes.c_int32), ("scale_den", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("clip", ctypes.c_float), ("eps", ctypes.c_float),
                ("features", ctypes.c_int32), ("precision", ctypes.c_int32), ("margin", ctypes.c_float),
                ("tune_feat_rows", ctypes.c_int32), ("tune_score_rows", ctypes.c_int32),
                ("tune_grid", ctypes.c_int32), ("prune_keep", ctypes.c_int32), ("pruner", ctypes.c_void_p)]

    TUNING = ("tune_feat_rows", "tune_score_rows", "tune_grid")

    def tuning(self) -> dict:
        return {k: int(getattr(self, k)) for k in self.TUNING}


class Level(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("h", ctypes.c_int32), ("pitch", ctypes.c_int32),
                ("cells_x", ctypes.c_int32), ("cells_y", ctypes.c_int32),
                ("blocks_x", ctypes.c_int32), ("blocks_y", ctypes.c_int32),
                ("win_x", ctypes.c_int32), ("win_y", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("offset", ctypes.c_int64)]


class NetMap(ctypes.Structure):
    _fields_ = [("cellmap", ctypes.c_void_p), ("logits", ctypes.c_void_p), ("labels", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("cells_x", ctypes.c_int32), ("cells_y", ctypes.c_int32)]


class Frame(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("w", ctypes.c_int32), ("h", ctypes.c_int32),
                ("pitch", ctypes.c_int32), ("reserved", ctypes.c_int32)]


BOX_DTYPE = np.dtype([("frame", "<i4"), ("level", "<i4"), ("i", "<i4"), ("j", "<i4"), ("model", "<i4"),
                      ("x0", "<i4"), ("y0", "<i4"), ("x1", "<i4"), ("y1", "<i4"),
                      ("score", "<f4"), ("score64", "<f8")])
COUNTS_DTYPE = np.dtype([("candidates", "<i4"), ("kept", "<i4"), ("overflow", "<i4"), ("rescored", "<i4")])
assert BOX_DTYPE.itemsize == 48 and COUNTS_DTYPE.itemsize == 16

_lib = None

_SIGS = {
    "pd_params_default": (None, [ctypes.c_void_p]),
    "pd_plan_pyramid": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_build_pyramid": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_lbp_codes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "pd_lbp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_void_p]),
    "pd_hog": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_void_p]),
    "pd_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_packed_models_bytes": (ctypes.c_int64, []),
    "pd_pack_models": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_score_windows_bf16": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "pd_detect_candidates": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "pd_lbp_blocks": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "pd_fold_lbp_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_lbp_naive": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "pd_lbp_scatter": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "pd_hog_global": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_score_windows_naive": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "pd_score_windows_wave": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "pd_score_windows": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "pd_detect_workspace_bytes": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]),
    "pd_detect": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_detect_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_graph_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "pd_graph_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pd_ctx_create": (ctypes.c_int, [ctypes.c_void_p]),
    "pd_ctx_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pd_ctx_detect": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "pd_ctx_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "pd_ctx_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_int, ctypes.c_void_p]),
    "pd_ctx_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.c_float]),
    "pd_ctx_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "pd_ctx_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "pd_pruner_save": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p]),
    "pd_pruner_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_video_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "pd_video_push": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double]),
    "pd_video_pop": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "pd_video_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pd_graph_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pd_graph_stage_ms": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pd_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "pd_features_cellmap": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "pd_pruner_workspace_bytes": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int]),
    "pd_pruner_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_void_p]),
    "pd_pruner_gradient": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_float,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p]),
    "pd_adam_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_void_p]),
    "pd_window_labels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_pruner_logits_bf16_workspace_bytes": (ctypes.c_int64, [ctypes.c_int, ctypes.c_int]),
    "pd_pruner_logits_bf16": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_void_p]),
    "pd_nms": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                              ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "pd_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "pd_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "pd_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pd_last_error": (ctypes.c_char_p, []),
    "pd_version": (ctypes.c_char_p, []),
}

EXPORTED = tuple(_SIGS)


def lib():
    """The loaded libpd (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_1611_01642_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != 0:
        raise PdError(rc, lib().pd_last_error().decode())


def params(scale=(11, 10), max_levels: int = 0, clip: float = 0.2, eps: float = 1e-3,
           features: int = FEAT_HOG | FEAT_LBP, precision: int = PREC_F32, margin: float = 0.05,
           tune_feat_rows: int = 0, tune_score_rows: int = 0, tune_grid: int = 0, prune_keep: int = 0,
           pruner=None) -> Params:
    """pd_params; `pruner` is a device float32 tensor of PRUNER_PARAMS values
    (the caller keeps it alive while the params are in use)."""
    p = Params()
    lib().pd_params_default(ctypes.byref(p))
    p.scale_num, p.scale_den = scale
    p.max_levels = max_levels
    p.clip = clip
    p.eps = eps
    p.features = features
    p.precision = precision
    p.margin = margin
    p.tune_feat_rows, p.tune_score_rows, p.tune_grid = tune_feat_rows, tune_score_rows, tune_grid
    p.prune_keep = prune_keep
    p.pruner = pruner.data_ptr() if pruner is not None else None
    return p


def plan_pyramid(w: int, h: int, prm: Params = None):
    """(levels, bytes): exact level sizes and packed offsets (host only)."""
    prm = prm or params()
    arr = (Level * MAX_LEVELS)()
    n = ctypes.c_int(0)
    nbytes = ctypes.c_int64(0)
    _check(lib().pd_plan_pyramid(w, h, ctypes.byref(prm), arr, MAX_LEVELS, ctypes.byref(n), ctypes.byref(nbytes)))
    return [arr[k] for k in range(n.value)], nbytes.value


# ---------------------------------------------------------------- device --

def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _image_args(img):
    torch = _torch()
    if img.dtype != torch.uint8 or img.dim() != 2 or not img.is_cuda or img.stride(1) != 1:
        raise ValueError("expected a 2-D uint8 CUDA tensor with unit column stride")
    h, w = img.shape
    return ctypes.c_void_p(img.data_ptr()), int(w), int(h), int(img.stride(0))


def build_pyramid(img, prm: Params = None):
    """(pyramid bytes, levels, views): all levels in one launch; `views` are
    [h][w] uint8 views into the packed buffer."""
    torch = _torch()
    p, w, h, pitch = _image_args(img)
    levels, nbytes = plan_pyramid(w, h, prm)
    pyr = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=img.device)
    arr = (Level * max(len(levels), 1))(*levels)
    _check(lib().pd_build_pyramid(p, w, h, pitch, arr, len(levels), ctypes.c_void_p(pyr.data_ptr()), _stream()))
    views = [pyr[L.offset:L.offset + L.pitch * L.h].view(L.h, L.pitch)[:, :L.w] for L in levels]
    return pyr, levels, views


def lbp_codes(img):
    torch = _torch()
    p, w, h, pitch = _image_args(img)
    out = torch.empty((h, w), dtype=torch.uint8, device=img.device)
    _check(lib().pd_lbp_codes(p, w, h, pitch, ctypes.c_void_p(out.data_ptr()), w, _stream()))
    return out


def features(img, prm: Params = None, hog: bool = True, lbp: bool = True, bf16: bool = False):
    """(blocks [36][Hb][Wb] float32 (bfloat16 if bf16) or None,
    cells [59][Hc][Wc] uint8 or None)."""
    torch = _torch()
    prm = prm or params()
    p, w, h, pitch = _image_args(img)
    hc, wc = h // CELL, w // CELL
    blocks = torch.empty((HOG_BLOCK, max(hc - 1, 0), max(wc - 1, 0)),
                         dtype=torch.bfloat16 if bf16 else torch.float32, device=img.device) if hog else None
    cells = torch.empty((LBP_BINS, hc, wc), dtype=torch.uint8, device=img.device) if lbp else None
    bptr = blocks.data_ptr() if hog else 0
    _check(lib().pd_features(p, w, h, pitch, ctypes.byref(prm),
                             ctypes.c_void_p(bptr if not bf16 else 0), ctypes.c_void_p(bptr if bf16 else 0),
                             ctypes.c_void_p(cells.data_ptr() if lbp else 0), _stream()))
    return blocks, cells


def pack_models(weights):
    """Packed BF16 hi/lo model buffer (uint8 device tensor) for score_windows_bf16."""
    torch = _torch()
    weights = weights.contiguous()
    out = torch.empty(int(lib().pd_packed_models_bytes()), dtype=torch.uint8, device=weights.device)
    _check(lib().pd_pack_models(ctypes.c_void_p(weights.data_ptr()), int(weights.shape[0]),
                                ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


def score_windows_bf16(blocks_bf16, cells, packed, bias, n_models: int):
    """Scores [m][Hc-15][Wc-7] float32 from BF16 HOG planes on BF16 MFMA."""
    torch = _torch()
    hc, wc = int(cells.shape[1]), int(cells.shape[2])
    if blocks_bf16.dtype != torch.bfloat16 or blocks_bf16.shape != (HOG_BLOCK, hc - 1, wc - 1):
        raise ValueError("blocks must be bfloat16 [36][Hc-1][Wc-1]")
    out = torch.empty((n_models, max(hc - 15, 0), max(wc - 7, 0)), dtype=torch.float32, device=cells.device)
    _check(lib().pd_score_windows_bf16(ctypes.c_void_p(blocks_bf16.data_ptr()), ctypes.c_void_p(cells.data_ptr()),
                                       wc, hc, ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(bias.data_ptr()),
                                       n_models, ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


def hog(img, prm: Params = None):
    return features(img, prm, hog=True, lbp=False)[0]


def lbp(img):
    return features(img, None, hog=False, lbp=True)[1]


def lbp_blocks(cells):
    """LBP block histograms (pd_lbp_blocks) of cell histograms uint8
    [59][Hc][Wc] or [n][59][Hc][Wc]: int16 [..][59][Hc-1][Wc-1] (counts up to
    256, held in int16 storage)."""
    torch = _torch()
    if cells.dtype != torch.uint8 or cells.dim() not in (3, 4) or not cells.is_contiguous():
        raise ValueError("cells must be contiguous uint8 [59][Hc][Wc] or [n][59][Hc][Wc]")
    c4 = cells if cells.dim() == 4 else cells.unsqueeze(0)
    n, _, hc, wc = (int(x) for x in c4.shape)
    out = torch.empty((n, LBP_BINS, max(hc - 1, 0), max(wc - 1, 0)), dtype=torch.int16, device=cells.device)
    _check(lib().pd_lbp_blocks(ctypes.c_void_p(c4.data_ptr()), n, hc, wc, ctypes.c_void_p(out.data_ptr()),
                               _stream()))
    return out if cells.dim() == 4 else out[0]


def fold_lbp_weights(wb):
    """The cell-level models [m][11332] (pd_fold_lbp_weights) with the same
    window scores as block-level models wb [m][9975] (HOG, then LBP block
    histograms)."""
    torch = _torch()
    wb = wb.contiguous()
    if wb.dtype != torch.float32 or wb.dim() != 2 or int(wb.shape[1]) != BLOCK_MODEL_DIM:
        raise ValueError("wb must be float32 [m][9975]")
    m = int(wb.shape[0])
    out = torch.empty((m, FEATURE_DIM), dtype=torch.float32, device=wb.device)
    _check(lib().pd_fold_lbp_weights(ctypes.c_void_p(wb.data_ptr()), m, ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


def score_windows(blocks, cells, weights, bias):
    """Scores [m][Hc-15][Wc-7] float32 of every window for every model."""
    torch = _torch()
    hc, wc = int(cells.shape[1]), int(cells.shape[2])
    if blocks.shape != (HOG_BLOCK, hc - 1, wc - 1) or not blocks.is_contiguous() or not cells.is_contiguous():
        raise ValueError("blocks must be [36][Hc-1][Wc-1] and cells [59][Hc][Wc], contiguous")
    weights = weights.contiguous()
    m = int(weights.shape[0])
    out = torch.empty((m, max(hc - 15, 0), max(wc - 7, 0)), dtype=torch.float32, device=cells.device)
    _check(lib().pd_score_windows(ctypes.c_void_p(blocks.data_ptr()), ctypes.c_void_p(cells.data_ptr()), wc, hc,
                                  ctypes.c_void_p(weights.data_ptr()), ctypes.c_void_p(bias.data_ptr()), m,
                                  ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


# ------------------------------------------- the paper's own mappings --
def lbp_naive(codes):
    """pd_lbp_naive: uint32 [Hc][Wc][59] cell histograms from an LBP map
    (uint8 [h][w] CUDA tensor, e.g. lbp_codes(img)), a thread per cell."""
    torch = _torch()
    p, w, h, pitch = _image_args(codes)
    out = torch.empty((h // CELL, w // CELL, LBP_BINS), dtype=torch.int32, device=codes.device)
    _check(lib().pd_lbp_naive(p, w, h, pitch, ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


def lbp_scatter(codes):
    """pd_lbp_scatter: the same histograms by global atomics (Algorithm 2)."""
    torch = _torch()
    p, w, h, pitch = _image_args(codes)
    out = torch.empty((h // CELL, w // CELL, LBP_BINS), dtype=torch.int32, device=codes.device)
    _check(lib().pd_lbp_scatter(p, w, h, pitch, ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


def hog_global(img, prm: Params = None, grad=None):
    """pd_hog_global: blocks [36][Hb][Wb] float32 by the paper's Global
    variant (gradients through global memory, a thread per block)."""
    torch = _torch()
    prm = prm or params()
    p, w, h, pitch = _image_args(img)
    if grad is None or grad.numel() < 2 * w * h:
        grad = torch.empty(2 * w * h, dtype=torch.float32, device=img.device)
    out = torch.empty((HOG_BLOCK, max(h // CELL - 1, 0), max(w // CELL - 1, 0)), dtype=torch.float32,
                      device=img.device)
    _check(lib().pd_hog_global(p, w, h, pitch, ctypes.byref(prm), ctypes.c_void_p(grad.data_ptr()),
                               ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


def _score_baseline(fn, blocks, cells, weights, bias):
    torch = _torch()
    hc, wc = int(cells.shape[1]), int(cells.shape[2])
    if blocks.shape != (HOG_BLOCK, hc - 1, wc - 1) or not blocks.is_contiguous() or not cells.is_contiguous():
        raise ValueError("blocks must be [36][Hc-1][Wc-1] and cells [59][Hc][Wc], contiguous")
    weights = weights.contiguous()
    m = int(weights.shape[0])
    out = torch.empty((m, max(hc - 15, 0), max(wc - 7, 0)), dtype=torch.float32, device=cells.device)
    _check(fn(ctypes.c_void_p(blocks.data_ptr()), ctypes.c_void_p(cells.data_ptr()), wc, hc,
              ctypes.c_void_p(weights.data_ptr()), ctypes.c_void_p(bias.data_ptr()), m,
              ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


def score_windows_naive(blocks, cells, weights, bias):
    """pd_score_windows_naive: a thread per window."""
    return _score_baseline(lib().pd_score_windows_naive, blocks, cells, weights, bias)


def score_windows_wave(blocks, cells, weights, bias):
    """pd_score_windows_wave: a wave per window (Algorithm 6)."""
    return _score_baseline(lib().pd_score_windows_wave, blocks, cells, weights, bias)


# ------------------------------------------------------------- pruner --
def features_cellmap(img, prm: Params = None):
    """(blocks [36][Hb][Wb] float32, cells [59][Hc][Wc] uint8, cell map
    [68][Hc][Wc] float32) of one level in one pass."""
    torch = _torch()
    prm = prm or params()
    p, w, h, pitch = _image_args(img)
    hc, wc = h // CELL, w // CELL
    blocks = torch.empty((HOG_BLOCK, max(hc - 1, 0), max(wc - 1, 0)), dtype=torch.float32, device=img.device)
    cells = torch.empty((LBP_BINS, hc, wc), dtype=torch.uint8, device=img.device)
    cmap = torch.empty((PRUNER_CHANNELS, hc, wc), dtype=torch.float32, device=img.device)
    _check(lib().pd_features_cellmap(p, w, h, pitch, ctypes.byref(prm), ctypes.c_void_p(blocks.data_ptr()),
                                     ctypes.c_void_p(cells.data_ptr()), ctypes.c_void_p(cmap.data_ptr()),
                                     _stream()))
    return blocks, cells, cmap


class PrunerBatch:
    """Device buffers of pd_pruner_forward / pd_pruner_gradient for a fixed
    list of cell maps ([68][Hc][Wc] float32 tensors) with optional labels and
    masks ([Hc][Wc] float32)."""

    def __init__(self, cellmaps, labels=None, masks=None, workspace=None):
        torch = _torch()
        self.cellmaps = [c.contiguous() for c in cellmaps]
        dev = self.cellmaps[0].device
        self.logits = [torch.empty((int(c.shape[1]), int(c.shape[2])), dtype=torch.float32, device=dev)
                       for c in self.cellmaps]
        self.labels, self.masks = labels, masks
        n = len(self.cellmaps)
        self._maps = (NetMap * n)()
        for k, c in enumerate(self.cellmaps):
            m = self._maps[k]
            m.cellmap, m.logits = c.data_ptr(), self.logits[k].data_ptr()
            m.labels = labels[k].data_ptr() if labels is not None else 0
            m.mask = masks[k].data_ptr() if masks is not None else 0
            m.cells_x, m.cells_y = int(c.shape[2]), int(c.shape[1])
        nbytes = int(lib().pd_pruner_workspace_bytes(self._maps, n))
        _check(nbytes if nbytes < 0 else 0)
        self.ws_bytes = nbytes
        if workspace is not None and workspace.numel() >= nbytes + 256:
            self.workspace = workspace  # shared by batches that run one after another
        else:
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        self.ws_ptr = self.workspace.data_ptr() + (-self.workspace.data_ptr()) % 256
        self.grad = torch.empty(PRUNER_PARAMS, dtype=torch.float32, device=dev)
        self.stats = torch.zeros(2, dtype=torch.float64, device=dev)

    def forward(self, weights):
        _check(lib().pd_pruner_forward(self._maps, len(self.cellmaps), ctypes.c_void_p(weights.data_ptr()),
                                       ctypes.c_void_p(self.ws_ptr), self.ws_bytes, _stream()))
        return self.logits

    def gradient(self, weights, pos_weight: float):
        """Enqueue forward + backward; self.grad and self.stats (loss, N) hold the results."""
        _check(lib().pd_pruner_gradient(self._maps, len(self.cellmaps), ctypes.c_void_p(weights.data_ptr()),
                                        float(pos_weight), ctypes.c_void_p(self.grad.data_ptr()),
                                        ctypes.c_void_p(self.stats.data_ptr()), ctypes.c_void_p(self.ws_ptr),
                                        self.ws_bytes, _stream()))
        return self.grad


def pruner_logits_bf16(img, weights, prm: Params = None):
    """Logits [Hc][Wc] float32 of one level by the BF16 MFMA inference path."""
    torch = _torch()
    prm = prm or params()
    p, w, h, pitch = _image_args(img)
    nbytes = int(lib().pd_pruner_logits_bf16_workspace_bytes(w, h))
    _check(nbytes if nbytes < 0 else 0)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=img.device)
    ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
    out = torch.empty((h // CELL, w // CELL), dtype=torch.float32, device=img.device)
    _check(lib().pd_pruner_logits_bf16(p, w, h, pitch, ctypes.byref(prm), ctypes.c_void_p(weights.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ptr), nbytes, _stream()))
    out._workspace = ws  # keep alive until the stream is done
    return out


def adam_step(params_, grad, m, v, step: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8) -> None:
    _check(lib().pd_adam_step(ctypes.c_void_p(params_.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                              ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), int(params_.numel()),
                              int(step), lr, beta1, beta2, eps, _stream()))


def pruner_save(path: str, params_, m, v, step: int, seed: int) -> None:
    """Checkpoint (pd_pruner_save): device float32 [PRUNER_PARAMS] parameters
    and Adam moments, the Adam step count and the training-order seed."""
    _check(lib().pd_pruner_save(os.fsencode(path), ctypes.c_void_p(params_.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                                ctypes.c_void_p(v.data_ptr()), int(step), int(seed), _stream()))


def pruner_load(path: str, params_, m=None, v=None):
    """Fills the device tensors from a checkpoint (pd_pruner_load); returns
    (step, seed)."""
    step, seed = ctypes.c_int64(0), ctypes.c_uint64(0)
    _check(lib().pd_pruner_load(os.fsencode(path), ctypes.c_void_p(params_.data_ptr()),
                                ctypes.c_void_p(m.data_ptr() if m is not None else 0),
                                ctypes.c_void_p(v.data_ptr() if v is not None else 0), ctypes.byref(step),
                                ctypes.byref(seed), _stream()))
    return int(step.value), int(seed.value)


def window_labels(scores, cells_x: int, cells_y: int, threshold):
    """(labels, mask) [Hc][Wc] float32 of one level from its window scores
    [Hc-15][Wc-7] (max over models) and a device float64 threshold [1]."""
    torch = _torch()
    scores = scores.contiguous()
    lab = torch.empty((cells_y, cells_x), dtype=torch.float32, device=scores.device)
    mask = torch.empty_like(lab)
    _check(lib().pd_window_labels(ctypes.c_void_p(scores.data_ptr()), int(scores.shape[1]), int(scores.shape[0]),
                                  cells_x, cells_y, ctypes.c_void_p(threshold.data_ptr()),
                                  ctypes.c_void_p(lab.data_ptr()), ctypes.c_void_p(mask.data_ptr()), _stream()))
    return lab, mask


def nms(cand_score, cand_key, level_wh, cap: int):
    """Greedy NMS of one frame's candidates.  cand_score: float32 [n] device;
    cand_key: int32 [n][4] (level, i, j, model) device; level_wh: host list of
    (w, h).  Returns (boxes uint8 [cap*48] device, counts uint8 [16] device)."""
    torch = _torch()
    n = int(cand_score.numel())
    wh = (ctypes.c_int32 * (2 * len(level_wh)))(*[v for pair in level_wh for v in pair])
    dev = cand_score.device
    boxes = torch.empty(max(cap, 1) * BOX_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    counts = torch.empty(COUNTS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    _check(lib().pd_nms(ctypes.c_void_p(cand_score.data_ptr()), ctypes.c_void_p(cand_key.data_ptr()), n, wh,
                        len(level_wh), ctypes.c_void_p(boxes.data_ptr()), cap,
                        ctypes.c_void_p(counts.data_ptr()), _stream()))
    return boxes, counts


def _frames_array(frames):
    arr = (Frame * len(frames))()
    for f, img in enumerate(frames):
        p, w, h, pitch = _image_args(img)
        arr[f].data, arr[f].w, arr[f].h, arr[f].pitch = p.value, w, h, pitch
    return arr


def workspace_bytes(sizes, n_models: int = 1, prm: Params = None) -> int:
    """Workspace bytes pd_detect needs for frames of these (w, h) sizes."""
    prm = prm or params()
    arr = (Frame * len(sizes))()
    for f, (w, h) in enumerate(sizes):
        arr[f].w, arr[f].h = w, h
    v = lib().pd_detect_workspace_bytes(arr, len(sizes), ctypes.byref(prm), n_models)
    if v < 0:
        _check(int(v))
    return int(v)


def detect_noalloc(frames, weights, bias, prm: Params, thresholds, boxes, counts, cap: int) -> None:
    """pd_detect_noalloc: the pipeline on the library's static scratch array
    (no workspace).  frames: uint8 CUDA tensors; boxes / counts: uint8 CUDA
    tensors of at least n * cap * 48 and n * 16 bytes."""
    arr = _frames_array(frames)
    weights = weights.contiguous()
    _check(lib().pd_detect_noalloc(arr, len(frames), ctypes.c_void_p(weights.data_ptr()),
                                   ctypes.c_void_p(bias.data_ptr()), int(weights.shape[0]), ctypes.byref(prm),
                                   ctypes.c_void_p(thresholds.data_ptr()), ctypes.c_void_p(boxes.data_ptr()), cap,
                                   ctypes.c_void_p(counts.data_ptr()), _stream()))


class Context:
    """A pd_ctx: the tuning table (per batch shape) and the graph cache of
    pd_ctx_detect.  Give it to Detectors (Detector(..., ctx=...)) so their
    run() and autotune() go through it."""

    def __init__(self):
        self.handle = ctypes.c_void_p(0)
        _check(lib().pd_ctx_create(ctypes.byref(self.handle)))

    def tuning(self, sizes, n_models: int, prm: Params):
        """params with the table's tuning fields for frames of these (w, h)
        sizes, or None when the table has no entry."""
        arr = (Frame * len(sizes))()
        for f, (w, h) in enumerate(sizes):
            arr[f].w, arr[f].h = w, h
        out = Params()
        rc = lib().pd_ctx_tuning(self.handle, arr, len(sizes), ctypes.byref(prm), n_models, ctypes.byref(out))
        if rc < 0:
            _check(rc)
        return out if rc == 1 else None

    def set_tuning(self, sizes, n_models: int, prm: Params, ms: float = 0.0) -> None:
        arr = (Frame * len(sizes))()
        for f, (w, h) in enumerate(sizes):
            arr[f].w, arr[f].h = w, h
        _check(lib().pd_ctx_set_tuning(self.handle, arr, len(sizes), ctypes.byref(prm), n_models, float(ms)))

    def save(self, path: str) -> None:
        _check(lib().pd_ctx_save(self.handle, os.fsencode(path)))

    def load(self, path: str) -> None:
        _check(lib().pd_ctx_load(self.handle, os.fsencode(path)))

    def close(self) -> None:
        if self.handle:
            h, self.handle = self.handle, ctypes.c_void_p(0)
            _check(lib().pd_ctx_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Detector:
    """Holds the device buffers of pd_detect for one batch shape; with a
    Context, run() and autotune() go through it (pd_ctx_detect,
    pd_ctx_autotune)."""
    frames: list
    weights: object
    bias: object
    prm: Params
    cap: int = 1024
    ctx: Context = None

    def __post_init__(self):
        torch = _torch()
        self.weights = self.weights.contiguous()
        self.n_models = int(self.weights.shape[0])
        self.sizes = [(int(f.shape[1]), int(f.shape[0])) for f in self.frames]
        self.ws_bytes = workspace_bytes(self.sizes, self.n_models, self.prm)
        dev = self.frames[0].device
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self.ws_ptr = self.workspace.data_ptr() + off
        n = len(self.frames)
        self.boxes = torch.empty(n * max(self.cap, 1) * BOX_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        self.counts = torch.empty(n * COUNTS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        self._frames = _frames_array(self.frames)

    def run(self, thresholds) -> None:
        """Enqueue the whole pipeline; thresholds: float64 CUDA tensor [n_frames]."""
        if self.ctx is not None:
            self._thr_ctx = thresholds  # a cached graph keeps reading this buffer
            _check(lib().pd_ctx_detect(self.ctx.handle, *self._args(thresholds), _stream()))
        else:
            _check(lib().pd_detect(*self._args(thresholds), _stream()))

    def _args(self, thresholds):
        return (self._frames, len(self.frames), ctypes.c_void_p(self.weights.data_ptr()),
                ctypes.c_void_p(self.bias.data_ptr()), self.n_models, ctypes.byref(self.prm),
                ctypes.c_void_p(thresholds.data_ptr()), ctypes.c_void_p(self.ws_ptr), self.ws_bytes,
                ctypes.c_void_p(self.boxes.data_ptr()), self.cap, ctypes.c_void_p(self.counts.data_ptr()))

    def capture(self, thresholds) -> None:
        """Capture the pipeline into a HIP graph (pd_graph_create).  The graph
        keeps the frame, weight and threshold buffers: refill them in place
        and call replay()."""
        self.release()
        self._thr_keep = thresholds
        h = ctypes.c_void_p(0)
        _check(lib().pd_graph_create(*self._args(thresholds), _stream(), ctypes.byref(h)))
        self._graph = h

    def replay(self) -> None:
        """Enqueue one launch of the captured graph on the current stream."""
        if getattr(self, "_graph", None) is None:
            raise RuntimeError("capture() first")
        _check(lib().pd_graph_launch(self._graph, _stream()))

    def release(self) -> None:
        g = getattr(self, "_graph", None)
        if g is not None:
            self._graph = None
            _check(lib().pd_graph_destroy(g))
        for h in getattr(self, "_steps", []):
            _check(lib().pd_graph_destroy(h))
        self._steps = []

    def capture_steps(self, thresholds, n: int) -> None:
        """n separate captures of the pipeline (replay_step(k)); captured
        while profile_enable(True) is on, each holds its own stage clock stamps,
        so step_stage_ms(k) gives replay k's stage times even when the n
        replays run back to back."""
        self.release()
        self._thr_keep = thresholds
        for _ in range(n):
            h = ctypes.c_void_p(0)
            _check(lib().pd_graph_create(*self._args(thresholds), _stream(), ctypes.byref(h)))
            self._steps.append(h)

    def replay_step(self, k: int) -> None:
        _check(lib().pd_graph_launch(self._steps[k], _stream()))

    def step_stage_ms(self, k: int) -> dict:
        """Per-stage GPU ms of the most recent replay of capture k."""
        ms = (ctypes.c_double * len(STAGES))()
        _check(lib().pd_graph_stage_ms(self._steps[k], ms))
        return dict(zip(STAGES, list(ms)))

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def autotune(self, thresholds, iters: int = 3):
        """Pick the tuning fields of the params by timing (pd_autotune); the
        detector keeps the result.  Returns (tuning dict, ms per call)."""
        best = Params()
        ms = ctypes.c_float(0.0)
        if self.ctx is not None:
            _check(lib().pd_ctx_autotune(self.ctx.handle, *self._args(thresholds), iters, ctypes.byref(best),
                                         ctypes.byref(ms), _stream()))
        else:
            _check(lib().pd_autotune(*self._args(thresholds), iters, ctypes.byref(best), ctypes.byref(ms),
                                     _stream()))
        self.prm = best
        return best.tuning(), float(ms.value)

    def candidates(self, frame: int):
        """(scores float32 [n], keys int32 [n][4], fp64 scores or None) of one
        frame's pre-NMS candidate list (after run(); n = candidates count)."""
        torch = _torch()
        counts = self.counts.cpu().numpy().view(COUNTS_DTYPE)
        n = int(counts[frame]["candidates"])
        dev = self.frames[0].device
        cs = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
        ck = torch.empty((max(n, 1), 4), dtype=torch.int32, device=dev)
        bf = self.prm.precision == PREC_BF16
        c64 = torch.empty(max(n, 1), dtype=torch.float64, device=dev) if bf else None
        _check(lib().pd_detect_candidates(self._frames, len(self.frames), ctypes.byref(self.prm), self.n_models,
                                          ctypes.c_void_p(self.ws_ptr), self.ws_bytes, frame,
                                          ctypes.c_void_p(cs.data_ptr()), ctypes.c_void_p(ck.data_ptr()),
                                          ctypes.c_void_p(c64.data_ptr() if bf else 0), n, _stream()))
        torch.cuda.synchronize()
        return (cs[:n].cpu().numpy(), ck[:n].cpu().numpy(), c64[:n].cpu().numpy() if bf else None)

    def results(self):
        """(boxes per frame as numpy structured arrays, counts structured array)."""
        counts = self.counts.cpu().numpy().view(COUNTS_DTYPE)
        allb = self.boxes.cpu().numpy().view(BOX_DTYPE).reshape(len(self.frames), max(self.cap, 1))
        return [allb[f, :counts[f]["kept"]].copy() for f in range(len(self.frames))], counts


class Video:
    """Streaming detection of host frames of one size (pd_video_*): push()
    queues a host uint8 frame with its threshold, pop() returns the oldest
    frame's (boxes, counts, device ms).  Up to `depth` frames in flight.
    The device weights and bias must outlive the video."""

    def __init__(self, w: int, h: int, weights, bias, prm: Params = None, cap: int = 1024, depth: int = 3):
        self.prm = prm or params()
        self.weights, self.bias = weights.contiguous(), bias.contiguous()
        self.w, self.h, self.cap = w, h, cap
        self.handle = ctypes.c_void_p(0)
        _check(lib().pd_video_create(w, h, ctypes.byref(self.prm), ctypes.c_void_p(self.weights.data_ptr()),
                                     ctypes.c_void_p(self.bias.data_ptr()), int(self.weights.shape[0]), cap, depth,
                                     ctypes.byref(self.handle)))
        self._boxes = np.zeros(cap, BOX_DTYPE)
        self._counts = np.zeros(1, COUNTS_DTYPE)

    def push(self, frame: np.ndarray, threshold: float) -> None:
        if frame.dtype != np.uint8 or frame.ndim != 2 or frame.shape[1] < self.w or frame.shape[0] < self.h:
            raise ValueError("frame must be a uint8 [h][>= w] host array")
        if frame.strides[1] != 1:
            raise ValueError("frame rows must be contiguous")
        _check(lib().pd_video_push(self.handle, ctypes.c_void_p(frame.ctypes.data), int(frame.strides[0]),
                                   float(threshold)))

    def pop(self):
        ms = ctypes.c_float(0.0)
        rc = lib().pd_video_pop(self.handle, ctypes.c_void_p(self._boxes.ctypes.data), self.cap,
                                ctypes.c_void_p(self._counts.ctypes.data), ctypes.byref(ms))
        if rc != E_OVERFLOW:  # a truncated frame is still a result: counts["overflow"] says so
            _check(rc)
        n = int(min(self._counts[0]["kept"], self.cap))
        return self._boxes[:n].copy(), self._counts[0].copy(), float(ms.value)

    def close(self) -> None:
        if self.handle:
            _check(lib().pd_video_destroy(self.handle))
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STAGES = ("upload", "zero", "resize", "features", "score", "compact", "nms")


def profile_enable(on: bool = True) -> None:
    """Record per-stage HIP events in later pd_detect calls of this thread."""
    _check(lib().pd_profile_enable(1 if on else 0))


def profile_read(reset: bool = True):
    """({stage: summed ms}, calls) over the recorded pd_detect calls."""
    ms = (ctypes.c_double * len(STAGES))()
    calls = ctypes.c_int64(0)
    _check(lib().pd_profile_read(ms, ctypes.byref(calls), 1 if reset else 0))
    return dict(zip(STAGES, list(ms))), calls.value


def decode_boxes(boxes_u8, counts_u8):
    counts = counts_u8.cpu().numpy().view(COUNTS_DTYPE)
    b = boxes_u8.cpu().numpy().view(BOX_DTYPE)
    return b[:counts[0]["kept"]].copy(), counts[0]
