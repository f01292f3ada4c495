"""Host-side checks of libpd's C ABI (no GPU work is launched here)."""
import ctypes
import os
import re

import pytest

import paper_1611_01642_amd as pd
from oracle import pd_oracle as O

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pd_[a-z0-9_]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    L = pd.lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(pd.EXPORTED)
    assert L.pd_version().decode().startswith("pd ")


def test_struct_sizes_match_header():
    assert ctypes.sizeof(pd.Params) == 56
    assert ctypes.sizeof(pd.Level) == 48
    assert ctypes.sizeof(pd.Frame) == 24
    assert pd.BOX_DTYPE.itemsize == 48


@pytest.mark.parametrize("w,h,scale,maxl", [
    (1242, 375, (11, 10), 0), (320, 240, (6, 5), 3), (320, 240, (6, 5), 0), (640, 480, (11, 10), 0),
    (1920, 1080, (11, 10), 0), (64, 128, (11, 10), 0), (63, 500, (11, 10), 0), (16384, 16384, (11, 10), 0),
    (16384, 3000, (101, 100), 0), (1000, 1000, (12, 10), 0), (777, 333, (3, 2), 2)])
def test_plan_matches_oracle_level_sizes(w, h, scale, maxl):
    levels, nbytes = pd.plan_pyramid(w, h, pd.params(scale=scale, max_levels=maxl))
    exp = O.level_sizes(w, h, scale[0], scale[1], maxl)[:pd.MAX_LEVELS]
    assert [(L.w, L.h) for L in levels] == exp
    off = 0
    for L in levels:
        assert L.pitch % 16 == 0 and L.pitch >= L.w and L.offset % 256 == 0 and L.offset >= off
        assert (L.cells_x, L.cells_y) == (L.w // 8, L.h // 8)
        assert (L.win_y, L.win_x) == O.window_grid(L.w, L.h)
        off = L.offset + L.pitch * L.h
    assert nbytes >= off


def test_plan_errors():
    L = pd.lib()
    n = ctypes.c_int()
    b = ctypes.c_int64()
    prm = pd.params()
    assert L.pd_plan_pyramid(0, 10, ctypes.byref(prm), None, 0, ctypes.byref(n), ctypes.byref(b)) == pd.E_SIZE
    assert L.pd_plan_pyramid(16385, 10, ctypes.byref(prm), None, 0, ctypes.byref(n), ctypes.byref(b)) == pd.E_SIZE
    bad = pd.params(scale=(10, 11))
    assert L.pd_plan_pyramid(100, 100, ctypes.byref(bad), None, 0, ctypes.byref(n), ctypes.byref(b)) == pd.E_ARG
    assert "scale" in L.pd_last_error().decode()
    assert L.pd_plan_pyramid(100, 100, None, None, 0, ctypes.byref(n), ctypes.byref(b)) == pd.E_ARG
    # an image smaller than a window is not an error: zero levels
    assert L.pd_plan_pyramid(50, 50, ctypes.byref(prm), None, 0, ctypes.byref(n), ctypes.byref(b)) == 0
    assert n.value == 0 and b.value == 0


def test_argument_errors_enqueue_nothing():
    L = pd.lib()
    prm = pd.params()
    nil = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the calls fail validation first
    assert L.pd_hog(nil, 64, 64, 64, ctypes.byref(prm), fake, nil) == pd.E_ARG
    assert L.pd_hog(fake, 64, 64, 32, ctypes.byref(prm), fake, nil) == pd.E_ARG  # pitch < width
    assert L.pd_hog(fake, 0, 64, 64, ctypes.byref(prm), fake, nil) == pd.E_SIZE
    assert L.pd_lbp(fake, 64, 64, 64, nil, nil) == pd.E_ARG
    assert L.pd_lbp_codes(fake, 20000, 64, 20000, fake, 20000, nil) == pd.E_SIZE
    bad = pd.params(features=4)
    assert L.pd_features(fake, 64, 64, 64, ctypes.byref(bad), fake, nil, fake, nil) == pd.E_ARG
    ok = pd.params()
    assert L.pd_features(fake, 64, 64, 64, ctypes.byref(ok), fake, fake, fake, nil) == pd.E_ARG  # FP32 and BF16
    assert L.pd_features(fake, 64, 64, 64, ctypes.byref(ok), nil, nil, nil, nil) == pd.E_ARG
    bad = pd.params(precision=7)
    assert L.pd_features(fake, 64, 64, 64, ctypes.byref(bad), fake, nil, fake, nil) == pd.E_ARG
    bad = pd.params(margin=-1.0)
    assert L.pd_features(fake, 64, 64, 64, ctypes.byref(bad), fake, nil, fake, nil) == pd.E_ARG
    assert L.pd_pack_models(fake, 9, fake, nil) == pd.E_SIZE
    assert L.pd_score_windows_bf16(fake, fake, 8, 16, fake, fake, 9, fake, nil) == pd.E_SIZE
    assert L.pd_score_windows_bf16(fake, fake, 7, 16, fake, fake, 1, fake, nil) == pd.E_SIZE
    # 8-model slices (HOG: 16 offset pairs x 8 chunks, LBP: 16 offsets x 15 chunks) + the 1-model fragments
    assert L.pd_packed_models_bytes() == ((16 * 8 + 16 * 15) * 16 * 32 + (8 + 2 * 15) * 64 * 8) * 2
    assert L.pd_score_windows(fake, fake, 7, 16, fake, fake, 1, fake, nil) == pd.E_SIZE
    assert L.pd_score_windows(fake, fake, 8, 16, fake, fake, 0, fake, nil) == pd.E_SIZE
    assert L.pd_score_windows(fake, fake, 8, 16, fake, fake, 17, fake, nil) == pd.E_SIZE
    assert L.pd_score_windows(nil, fake, 8, 16, fake, fake, 1, fake, nil) == pd.E_ARG
    wh = (ctypes.c_int32 * 2)(1242, 375)
    assert L.pd_nms(fake, fake, 4097, wh, 1, fake, 10, fake, nil) == pd.E_SIZE
    assert L.pd_nms(fake, fake, 10, wh, 0, fake, 10, fake, nil) == pd.E_SIZE
    assert L.pd_build_pyramid(fake, 100, 100, 100, nil, 65, fake, nil) == pd.E_SIZE
    assert L.pd_lbp_blocks(fake, 1, 1, 8, fake, nil) == pd.E_SIZE      # no block in one cell row
    assert L.pd_lbp_blocks(fake, 0, 16, 8, fake, nil) == pd.E_SIZE
    assert L.pd_lbp_blocks(fake, 1, 16, 2049, fake, nil) == pd.E_SIZE  # wider than PD_MAX_DIM
    assert L.pd_lbp_blocks(nil, 1, 16, 8, fake, nil) == pd.E_ARG
    assert L.pd_fold_lbp_weights(fake, 0, fake, nil) == pd.E_SIZE
    assert L.pd_fold_lbp_weights(fake, 17, fake, nil) == pd.E_SIZE
    assert L.pd_fold_lbp_weights(fake, 1, nil, nil) == pd.E_ARG
    out = ctypes.c_void_p(0)
    prm = pd.params()
    assert L.pd_video_create(640, 480, ctypes.byref(prm), fake, fake, 1, 16, 0, ctypes.byref(out)) == pd.E_SIZE
    assert L.pd_video_create(640, 480, ctypes.byref(prm), fake, fake, 1, 16, 17, ctypes.byref(out)) == pd.E_SIZE
    assert L.pd_video_create(640, 480, ctypes.byref(prm), fake, fake, 1, 0, 2, ctypes.byref(out)) == pd.E_SIZE
    assert L.pd_video_create(640, 480, ctypes.byref(prm), nil, fake, 1, 16, 2, ctypes.byref(out)) == pd.E_ARG
    assert L.pd_video_create(640, 480, ctypes.byref(prm), fake, fake, 1, 16, 2, nil) == pd.E_ARG
    assert not out.value
    assert L.pd_video_push(nil, fake, 640, 0.0) == pd.E_ARG
    assert L.pd_video_pop(nil, fake, 1, fake, nil) == pd.E_ARG
    assert L.pd_video_destroy(nil) == 0


def test_tuning_field_checks_and_graph_handles():
    L = pd.lib()
    fake = ctypes.c_void_p(0x1000)
    nil = ctypes.c_void_p(0)
    for kw in (dict(tune_feat_rows=3), dict(tune_feat_rows=33), dict(tune_score_rows=12), dict(tune_score_rows=2),
               dict(tune_grid=-1)):
        bad = pd.params(**kw)
        assert L.pd_features(fake, 64, 64, 64, ctypes.byref(bad), fake, nil, fake, nil) == pd.E_ARG, kw
        assert "tune" in L.pd_last_error().decode()
    for kw in (dict(tune_feat_rows=4), dict(tune_feat_rows=32), dict(tune_score_rows=16), dict(tune_grid=1)):
        assert pd.workspace_bytes([(1242, 375)], 2, pd.params(**kw)) == pd.workspace_bytes([(1242, 375)], 2)
    assert L.pd_graph_destroy(nil) == 0
    assert L.pd_graph_launch(nil, nil) == pd.E_ARG
    ms = (ctypes.c_double * len(pd.STAGES))()
    assert L.pd_graph_stage_ms(nil, ms) == pd.E_ARG
    arr = (pd.Frame * 1)()
    arr[0].data, arr[0].w, arr[0].h, arr[0].pitch = 0x1000, 100, 100, 100
    prm = pd.params()
    assert L.pd_graph_create(arr, 1, fake, fake, 1, ctypes.byref(prm), fake, fake, 16, fake, 10, fake, nil,
                             nil) == pd.E_ARG
    best = pd.Params()
    assert L.pd_autotune(arr, 1, fake, fake, 1, ctypes.byref(prm), fake, fake, 16, fake, 10, fake, 0,
                         ctypes.byref(best), nil, nil) == pd.E_ARG
    assert L.pd_autotune(arr, 1, fake, fake, 1, ctypes.byref(prm), fake, fake, 16, fake, 10, fake, 1,
                         ctypes.byref(best), nil, nil) == pd.E_WORKSPACE


def test_bf16_workspace_and_model_limit():
    prm = pd.params(precision=pd.PREC_BF16)
    assert pd.workspace_bytes([(1242, 375)], 8, prm) > 0
    L = pd.lib()
    arr = (pd.Frame * 1)()
    arr[0].w, arr[0].h = 1242, 375
    assert L.pd_detect_workspace_bytes(arr, 1, ctypes.byref(prm), 9) == pd.E_SIZE
    assert L.pd_detect_workspace_bytes(arr, 1, ctypes.byref(pd.params()), 9) > 0


def test_detect_workspace_and_errors():
    L = pd.lib()
    prm = pd.params()
    ws1 = pd.workspace_bytes([(1242, 375)])
    ws2 = pd.workspace_bytes([(1242, 375)] * 2)
    assert 0 < ws1 < ws2 < 3 * ws1
    # HOG FP32 + LBP u8 + scores of every level fit in the workspace
    levels, _ = pd.plan_pyramid(1242, 375, prm)
    feat = sum(36 * L_.blocks_x * L_.blocks_y * 4 + 59 * L_.cells_x * L_.cells_y + 4 * L_.win_x * L_.win_y
               for L_ in levels)
    assert ws1 > feat
    arr = (pd.Frame * 1)()
    arr[0].w, arr[0].h = 0, 10
    assert L.pd_detect_workspace_bytes(arr, 1, ctypes.byref(prm), 1) == pd.E_SIZE
    arr[0].w, arr[0].h = 100, 100
    assert L.pd_detect_workspace_bytes(arr, 1, ctypes.byref(prm), 0) == pd.E_SIZE
    fake = ctypes.c_void_p(0x1000)
    arr[0].data, arr[0].pitch = 0x1000, 100
    # workspace too small -> PD_E_WORKSPACE before any GPU work
    rc = L.pd_detect(arr, 1, fake, fake, 1, ctypes.byref(prm), fake, fake, 16, fake, 10, fake, ctypes.c_void_p(0))
    assert rc == pd.E_WORKSPACE
    arr[0].data = 0
    rc = L.pd_detect(arr, 1, fake, fake, 1, ctypes.byref(prm), fake, fake, 1 << 30, fake, 10, fake, ctypes.c_void_p(0))
    assert rc == pd.E_ARG
    # every error below is found on the host before any GPU work
    arr[0].data = 0x1000

    def detect(n=1, cap=10):
        return L.pd_detect(arr, n, fake, fake, 1, ctypes.byref(prm), fake, fake, 1 << 30, fake, cap, fake,
                           ctypes.c_void_p(0))
    assert detect(n=0) == pd.E_ARG        # an empty batch
    assert detect(cap=-1) == pd.E_ARG
    arr[0].w, arr[0].h, arr[0].pitch = 16385, 100, 16400
    assert detect() == pd.E_SIZE          # wider than PD_MAX_DIM
    arr[0].w, arr[0].h, arr[0].pitch = 100, 100, 99
    assert detect() == pd.E_ARG           # pitch below the width


def test_noalloc_rejects_batches_beyond_its_scratch_before_any_gpu_work():
    """pd_detect_noalloc checks the batch's workspace against the static
    scratch (PD_NOALLOC_SCRATCH_BYTES) on the host, before any HIP call."""
    L = pd.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced
    frames = (pd.Frame * 2)()
    for f in frames:
        f.data, f.w, f.h, f.pitch = 0x1000, 1920, 1080, 1920
    assert pd.workspace_bytes([(1920, 1080)] * 2) > pd.NOALLOC_SCRATCH_BYTES
    rc = L.pd_detect_noalloc(frames, 2, fake, fake, 1, ctypes.byref(pd.params()), fake, fake, 16, fake, None)
    assert rc == pd.E_WORKSPACE and "static scratch" in L.pd_last_error().decode()
    assert L.pd_detect_noalloc(frames, 0, fake, fake, 1, ctypes.byref(pd.params()), fake, fake, 16, fake,
                               None) == pd.E_ARG


def test_pruner_load_rejects_bad_files_before_any_gpu_work(tmp_path):
    """pd_pruner_load validates size, magic and checksum on the host before
    any copy: a missing, truncated or corrupted file is PD_E_IO."""
    L = pd.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced
    step, seed = ctypes.c_int64(0), ctypes.c_uint64(0)

    def load(path):
        return L.pd_pruner_load(os.fsencode(str(path)), fake, fake, fake, ctypes.byref(step), ctypes.byref(seed),
                                None)
    assert load(tmp_path / "missing") == pd.E_IO
    n = 32 + 3 * 4 * pd.PRUNER_PARAMS + 8
    good_size = bytearray(b"PDPRUNE1") + bytearray(n - 8)
    (tmp_path / "short").write_bytes(bytes(good_size[:-1]))
    assert load(tmp_path / "short") == pd.E_IO and "size" in L.pd_last_error().decode()
    bad = bytearray(good_size)
    bad[0:8] = b"NOTPRUNE"
    (tmp_path / "magic").write_bytes(bytes(bad))
    assert load(tmp_path / "magic") == pd.E_IO and "magic" in L.pd_last_error().decode()
    ok = bytearray(good_size)
    ok[8:12] = (1).to_bytes(4, "little")
    ok[12:16] = pd.PRUNER_PARAMS.to_bytes(4, "little")
    (tmp_path / "sum").write_bytes(bytes(ok))  # checksum left at zero
    assert load(tmp_path / "sum") == pd.E_IO and "checksum" in L.pd_last_error().decode()
    assert L.pd_pruner_load(None, fake, fake, fake, ctypes.byref(step), ctypes.byref(seed), None) == pd.E_ARG


def test_tuning_table_round_trip(tmp_path):
    ctx = pd.Context()
    sizes = [(1242, 375)] * 4 + [(640, 480)]
    assert ctx.tuning(sizes, 1, pd.params()) is None
    ctx.set_tuning(sizes, 1, pd.params(tune_feat_rows=12, tune_score_rows=4, tune_grid=512), 3.25)
    ctx.set_tuning(sizes, 8, pd.params(precision=pd.PREC_BF16, tune_feat_rows=10), 7.0)
    got = ctx.tuning(sizes, 1, pd.params())
    assert got.tuning() == {"tune_feat_rows": 12, "tune_score_rows": 4, "tune_grid": 512}
    assert ctx.tuning(sizes[:4], 1, pd.params()) is None            # another batch shape
    assert ctx.tuning(sizes, 1, pd.params(features=pd.FEAT_HOG)) is None
    path = str(tmp_path / "tuning.txt")
    ctx.save(path)
    other = pd.Context()
    other.load(path)
    assert other.tuning(sizes, 1, pd.params()).tuning() == got.tuning()
    assert other.tuning(sizes, 8, pd.params(precision=pd.PREC_BF16)).tune_feat_rows == 10
    text = open(path).read().splitlines()
    assert text[0] == "pd-tuning 1" and len(text) == 3
    (tmp_path / "bad.txt").write_text("pd-tuning 1\nshape\t99 4 0 1.0\n")
    with pytest.raises(pd.PdError) as e:
        other.load(str(tmp_path / "bad.txt"))
    assert e.value.code == pd.E_IO
    with pytest.raises(pd.PdError):
        other.tuning([(0, 10)], 1, pd.params())
