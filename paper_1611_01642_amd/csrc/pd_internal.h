// Internal declarations shared by the libpd HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pd.h"

namespace pd {

// Everything one kernel needs to know about one (frame, level) pair.  In a
// batched launch these live in a device table; single-level entry points
// pass one by value.
struct LevelItem {
    const uint8_t* src;   // level-0 image of the frame
    uint8_t* pyr;         // this level inside the pyramid buffer
    float* hog;           // [36][hb][wb] FP32, or NULL
    uint16_t* hog16;      // [36][hb][wb] BF16, or NULL
    uint8_t* lbp;         // [59][hc][wc]
    float* scores;        // [n_models][ny][nx]
    float* cmap;          // pruner cell map [68][hc][wc] FP32, or NULL
    uint16_t* cmap16;     // pruner cell map [hc][wc][72] BF16 (channels 68..71 zero), or NULL
    uint16_t* act1;       // pruner layer outputs [hc][wc][32] BF16
    uint16_t* act2;
    float* logit;         // pruner logits [hc][wc]
    int64_t cand_off;     // the frame's first entry in the candidate lists
    int32_t cand_cap;     // entries the frame owns there: its window count
    int32_t src_w, src_h, src_pitch;
    int32_t w, h, pitch;
    int32_t wc, hc, wb, hb, nx, ny;
    int32_t frame, level;
};

// ---- learned window pruner ----------------------------------------------
constexpr int PRUNER_CH[4] = {68, 32, 32, 16};  // cell-map channels, conv outputs
constexpr int PRUNER_WIN_DI = 7, PRUNER_WIN_DJ = 3;  // window (i, j) <-> cell (i + 7, j + 3)
constexpr int PRUNER_PARAMS = 68 * 32 * 9 + 32 + 32 * 32 * 9 + 32 + 32 * 16 * 9 + 16 + 16 + 1;
// buffer slots of a NetItem
enum { NET_X = 0, NET_A1, NET_A2, NET_A3, NET_GA, NET_GB, NET_SLOTS };

// One map (pyramid level) of a pruner launch: planar FP32 buffers.
struct NetItem {
    float* buf[NET_SLOTS];  // cell map (68), a1 (32), a2 (32), a3 (16), gradient buffers (32, 32)
    float* logit;           // [hc][wc]
    const float* label;     // [hc][wc] (training)
    const float* mask;      // [hc][wc] (training)
    int32_t wc, hc;
};

// One workgroup's share of a batched launch: which item and which tile.
// FP32 scoring tiles keep the model in pad's low 16 bits and the lane-group
// width (64, 32 or 16 window columns) in its high bits.
struct Tile {
    int32_t item;
    int32_t ty, tx;
    int32_t pad;
};
__host__ __device__ inline int tile_model(const Tile& t) { return t.pad & 0xffff; }
__host__ __device__ inline int tile_width(const Tile& t) {
    const int w = t.pad >> 16;
    return w ? w : 64;
}
__host__ __device__ inline int32_t score_pad(int model, int width) { return model | ((width == 64 ? 0 : width) << 16); }

// Greedy-NMS geometry of one frame: sizes of its levels, level 0 first, and
// where its candidate list lives.  A frame's candidate list holds one entry
// per window at most, so it is sized by the frame's window count and never
// drops a candidate; NMS takes the PD_MAX_CANDIDATES highest-scoring ones.
struct NmsGeom {
    int32_t n_levels;
    int32_t cand_cap;  // the frame's window count
    int64_t cand_off;  // first entry of the frame's candidate list
    int32_t wh[PD_MAX_LEVELS][2];
};

// XCDs (chiplets with their own L2) that workgroups are dealt to, round-robin
constexpr int N_XCD = 8;

// ---- tile shapes ---------------------------------------------------------
// resize: 64 lanes x 4 pixels wide, 16 rows
constexpr int RS_TX = 256;      // pixels per tile row
constexpr int RS_TY = 16;       // rows per tile (single-image launches; the least in tables)
constexpr int RS_TY_MAX = 128;  // rows per tile in tables
constexpr int RS_LDS = 20 * 1024;  // staged source bytes per resize workgroup (7 workgroups per CU)
// features: one wave = a strip of 64 cell columns (one per lane) walking
// down FT_CH block rows (+1 overlap cell row); it owns 63 block columns
constexpr int FT_W = 64;
constexpr int FT_BX = 63;
constexpr int FT_CH = 8;
constexpr int FT_WAVES = 4;  // waves (independent strips) per workgroup
// scoring: one wave = 64 window columns x SC_R window rows
constexpr int SC_R = 8;
constexpr int SC_W = 64;
constexpr int SC_WAVES = 4;  // waves (independent tiles) per workgroup
// compaction: threads per workgroup, windows per thread, windows per workgroup
constexpr int CP_THREADS = 256;
constexpr int CP_PER = 4;
constexpr int CP_N = CP_THREADS * CP_PER;
// MFMA scoring tile: window rows x window columns
constexpr int MF_TILE_R = 4;
constexpr int MF_TILE_C = 64;

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// ---- uniform LBP table (Section 4.2) -----------------------------------------
// Codes with at most two circular 0/1 transitions take bins 0..57 in ascending
// code order; all others share bin 58.  Each kernel source that needs it
// places its own __constant__ copy (make_lbp_table() at compile time).
struct LbpTable {
    uint8_t bin[256];
};

constexpr int popcount8(int v) {
    int n = 0;
    for (int k = 0; k < 8; ++k) n += (v >> k) & 1;
    return n;
}

constexpr LbpTable make_lbp_table() {
    LbpTable t{};
    int next = 0;
    for (int c = 0; c < 256; ++c) {
        const int rot = ((c >> 1) | (c << 7)) & 255;  // rotate right by one bit
        t.bin[c] = (uint8_t)(popcount8(c ^ rot) <= 2 ? next++ : 58);
    }
    return t;
}

// Device buffers reached through tables in memory (LevelItem and the like)
// are typed as global memory inside kernels: the compiler cannot infer the
// address space of such pointers and would emit FLAT accesses, which also
// count against the LDS wait counter and so stall LDS reads behind prefetches.
// (The host pass of the same source sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <typename T>
using gptr = T*;
#endif
template <typename T>
__device__ __forceinline__ gptr<T> gmem(T* p) {
    return (gptr<T>)p;
}

// Raw buffer view of `bytes` bytes at `base` (a level's feature planes, at
// most 4 GiB): loads take a 32-bit lane offset and a wave-uniform byte offset
// in a scalar register, with no per-value address arithmetic; a read past
// `bytes` returns 0 instead of faulting.  Word 3 is the gfx9 raw-buffer format.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t planes_rsrc(const void* base, uint64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0,
                                             (int)(uint32_t)(bytes < 0xffffffffull ? bytes : 0xffffffffull),
                                             0x00020000);
}

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline int resize_tiles_x(int w) { return ceil_div(w, RS_TX); }
__host__ __device__ inline int resize_tiles_y(int h) { return ceil_div(h, RS_TY); }
// Rows per resize tile of a w x h level sampled from a sw x sh image: as many
// (a multiple of 4, RS_TY..RS_TY_MAX) as keep the tile's source rectangle
// within the staging buffer, so that levels near full scale run few, tall tiles.
inline int resize_rows(int w, int h, int sw, int sh) {
    const double sx = (double)sw / w, sy = (double)sh / h;
    const double row_bytes = (RS_TX - 1) * sx + 12.0;  // source span of a tile row + alignment slack
    const double src_rows = RS_LDS / row_bytes - 3.0;
    int rows = (int)(src_rows / sy) + 1;
    rows = rows / 4 * 4;
    return rows < RS_TY ? RS_TY : (rows > RS_TY_MAX ? RS_TY_MAX : rows);
}
__host__ __device__ inline int feat_tiles_x(int wc) { return wc <= 1 ? 1 : ceil_div(wc - 1, FT_BX); }
// Strips that also emit the pruner cell map own 62 columns: every owned cell
// needs both neighbours in the same wave.
constexpr int FT_BX_CM = 62;
__host__ __device__ inline int feat_tiles_x_cm(int wc) { return ceil_div(wc, FT_BX_CM); }
__host__ __device__ inline int feat_tiles_y(int hc, int rows = FT_CH) { return hc <= 1 ? 1 : ceil_div(hc - 1, rows); }
__host__ __device__ inline int score_tiles_x(int nx) { return ceil_div(nx, SC_W); }
__host__ __device__ inline int score_tiles_y(int ny, int rows = SC_R) { return ceil_div(ny, rows); }

// Tile shapes and launch shapes chosen at run time (pd_params tuning fields).
struct Tuning {
    int feat_rows = FT_CH;   // block rows per feature strip (2..32)
    int score_rows = SC_R;   // FP32 scoring: window rows per band (4, 8 or 16)
    int grid = 0;            // 0: one workgroup per tile group; > 0: at most this many, looping
};

// ---- launchers (each defined next to its kernel) ---------------------------
hipError_t launch_resize_single(const LevelItem* items, int n_items, hipStream_t s);
hipError_t launch_resize_table(const LevelItem* items, const Tile* tiles, int n_tiles, hipStream_t s);

hipError_t launch_lbp_codes(const uint8_t* img, int w, int h, int pitch, uint8_t* codes,
                            int codes_pitch, hipStream_t s);
hipError_t launch_features_single(const LevelItem& it, int features, float clip, float eps,
                                  hipStream_t s);
hipError_t launch_features_table(const LevelItem* items, const Tile* tiles, int n_tiles,
                                 int features, float clip, float eps, const Tuning& tu, hipStream_t s);
// Fused HOG + LBP + pruner cell map (it.cmap), HOG|LBP only.
hipError_t launch_features_cellmap_single(const LevelItem& it, float clip, float eps, hipStream_t s);
hipError_t launch_features_cellmap_table(const LevelItem* items, const Tile* tiles, int n_tiles, float clip,
                                         float eps, const Tuning& tu, hipStream_t s);

hipError_t launch_score_single(const LevelItem& it, const float* w, const float* bias, int n_models,
                               int features, hipStream_t s);
// FP32 scoring on the matrix cores (score32.hip): bands of window rows over
// runs of 16-column tiles, in 8 lists (one per XCD) taken through counters.
struct XcdLists {
    int32_t start[9];
};
constexpr int S32_COUNTERS = 8 * PD_MAX_MODELS;  // per model and XCD
int64_t score32_packed_floats(int n_models);
// Builds the band table of `rows` window rows (4, 8 or 16) into out (room for
// the sum of score32_band_capacity over the items); returns its entry count.
int score32_bands(const LevelItem* items, int n_items, int rows, int grid_cap, Tile* out, XcdLists* xs, int* grid);
int64_t score32_band_capacity(int nx, int ny, int wc);
hipError_t launch_pack_score32(const float* w, int n_models, float* out, hipStream_t s);
// Threshold decisions taken as the FP32 scores are stored (one model, no
// keep set): windows above their frame's threshold are appended to the
// frame's candidate list as compaction appends them.  counters NULL: none.
struct Decide32 {
    const double* thr;   // per frame
    int32_t* counters;   // per frame, zeroed: candidates appended
    float* cscore;       // candidate lists (LevelItem::cand_off, cand_cap)
    int4* ckey;
};
// ctr: S32_COUNTERS zeroed ints
hipError_t launch_score32_table(const LevelItem* items, const Tile* bands, const XcdLists& xs, int grid,
                                const float* packed, const float* bias, int n_models, int features, int rows,
                                int* ctr, const Decide32& dec, hipStream_t s);

// Error reporting of the C ABI: sets the calling thread's message and
// returns `code` (fail) or maps a HIP status (hip_status: PD_OK or PD_E_HIP).
int fail(int code, const char* fmt, ...);
int hip_status(hipError_t e, const char* what);
// Whether pd_profile_enable is on for the calling thread.
bool profiling_on();

hipError_t launch_lbp_blocks(const uint8_t* cells, int n, int hc, int wc, uint16_t* blocks, hipStream_t s);
hipError_t launch_fold_lbp_weights(const float* wb, int n_models, float* w, hipStream_t s);

int64_t packed_weight_elems();
int64_t rowgemm_packed_elems();
hipError_t launch_pack_rowgemm(const float* w, uint16_t* out, hipStream_t s);
hipError_t launch_rowgemm_single(const LevelItem& it, const uint16_t* packed, const float* bias, hipStream_t s);
hipError_t launch_rowgemm_table(const LevelItem* items, const Tile* tiles, int n_tiles, const uint16_t* packed,
                                const float* bias, int grid, hipStream_t s);
// row-GEMM scoring (one model): tile = 64 window columns, all rows
constexpr int RG_TILE_C = 64;
hipError_t launch_pack_weights(const float* w, int n_models, uint16_t* out, hipStream_t s);
hipError_t launch_mfma_single(const LevelItem& it, const uint16_t* wpk, const float* bias, int n_models, int features,
                              hipStream_t s);
hipError_t launch_mfma_table(const LevelItem* items, const Tile* tiles, int n_tiles, const uint16_t* wpk,
                             const float* bias, int n_models, int features, int grid, hipStream_t s,
                             const int* n_dev = nullptr);
// Windows with |score - threshold| < margin go to the near list (margin <= 0:
// none), whose capacity near_cap is the batch's window count, so no near
// window is ever dropped.  kth (optional): per frame, the K-th largest window
// logit of the pruner; only windows whose logit reaches it can be candidates.
hipError_t launch_compact(const LevelItem* items, const Tile* tiles, int n_tiles, int n_models,
                          const double* thresholds, float margin, int32_t* counters, float* cand_score,
                          int4* cand_key, double* cand_s64, int32_t* near_count, int4* near_key, int64_t near_cap,
                          int n_frames, const float* kth, hipStream_t s);
// near_count[n_frames] is the length of the dense near list near_key
// (entries: frame * PD_MAX_LEVELS + level, i, j, model)
// Gradient table of the FP64 rescore: entry dy * ORIENT_W + dx + 255 (dy in
// 0..255, dx in -255..255) holds (orientation bin coordinate, magnitude).
constexpr int ORIENT_W = 511, ORIENT_H = 256;
constexpr int64_t ORIENT_BYTES = (int64_t)ORIENT_W * ORIENT_H * 16;
hipError_t launch_orient_table(double2* table, hipStream_t s);
// features: PD_FEAT_HOG | PD_FEAT_LBP subset; the dot products run over
// that family's features only (the other family's weights are not read).
hipError_t launch_rescore64(const LevelItem* items, const int32_t* frame_first_item, int n_frames,
                            const int32_t* near_count, const int4* near_key, const float* weights,
                            const float* bias, int n_models, int features, float clip, float eps,
                            const double* thresholds, int32_t* counters, float* cand_score, int4* cand_key,
                            double* cand_s64, const double2* orient, hipStream_t s);
// Per frame whose candidate list is longer than PD_MAX_CANDIDATES: the
// PD_MAX_CANDIDATES entries with the smallest NMS sort keys (score
// descending, then level, i, j ascending) copied to the frame's slot of the
// sel_* arrays ([n_frames][PD_MAX_CANDIDATES]).  Other frames are left alone.
hipError_t launch_cand_select(const NmsGeom* geoms, int n_frames, const int32_t* counters, const float* cand_score,
                              const int4* cand_key, const double* cand_s64, float* sel_score, int4* sel_key,
                              double* sel_s64, hipStream_t s);
// NMS per frame over its candidate list, or over its sel_* slot when the
// list is longer than PD_MAX_CANDIDATES.
hipError_t launch_nms_table(const NmsGeom* geoms, int n_frames, const int32_t* counters,
                            const float* cand_score, const int4* cand_key, const double* cand_s64,
                            const float* sel_score, const int4* sel_key, const double* sel_s64,
                            const int32_t* near_count, pd_box* boxes, int cap, pd_counts* counts, hipStream_t s);
hipError_t launch_nms_single(const NmsGeom& g, int n, const float* cand_score, const int4* cand_key,
                             pd_box* boxes, int cap, pd_counts* counts, hipStream_t s);
// BF16 MFMA inference of the pruner network (channels-last BF16 maps).
constexpr int PR_CP1 = 72;  // layer-1 input channel stride
int64_t pruner_packed_bf16_elems();
hipError_t launch_pruner_pack_bf16(const float* params, uint16_t* packed, hipStream_t s);
int pruner_mfma_tiles_y(int hc);  // row pairs
// Per frame, the K-th largest window logit (-inf when K >= windows).
hipError_t launch_topk(const LevelItem* items, const int32_t* first_item, const NmsGeom* geoms, int n_frames,
                       int keep_k, float* kth, hipStream_t s);
// Appends the score tiles (rows x cols windows) that hold a kept window.
hipError_t launch_tile_filter(const LevelItem* items, const Tile* tiles, int n_tiles, int rows, int cols,
                              const float* kth, Tile* kept, int32_t* kept_count, hipStream_t s);
hipError_t launch_pruner_mfma(const LevelItem* items, const Tile* tiles, int n_tiles, const float* params,
                              const uint16_t* packed, hipStream_t s);
int64_t pruner_prep_floats();
hipError_t launch_pruner_prep(const float* params, float* prep, hipStream_t s);
hipError_t launch_pruner_forward(const NetItem* items, const Tile* tiles, int n_tiles, const float* params,
                                 const float* prep, bool keep_a3, hipStream_t s);
int pruner_wgrad_blocks(int n_tiles);
int64_t pruner_partial_floats(int n_tiles);
hipError_t launch_pruner_backward(const NetItem* items, const Tile* tiles, int n_tiles, const float* params,
                                  const float* prep, float pos_weight, float* grad, double* stats, float* partial,
                                  hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, int step, float lr, float b1, float b2,
                       float eps, hipStream_t s);
hipError_t launch_window_labels(const float* scores, int nx, int ny, int wc, int hc, const double* thr,
                                float* labels, float* mask, hipStream_t s);

hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t s);

// The paper's own mappings, as ablation baselines (baselines.hip).
hipError_t launch_lbp_naive(const uint8_t* codes, int pitch, int wc, int hc, uint32_t* hist, hipStream_t s);
hipError_t launch_lbp_scatter(const uint8_t* codes, int pitch, int wc, int hc, uint32_t* hist, hipStream_t s);
hipError_t launch_hog_global(const uint8_t* img, int w, int h, int pitch, float clip, float eps, float* grad,
                             float* blocks, hipStream_t s);
hipError_t launch_svm_naive(const float* blocks, const uint8_t* cells, int wc, int hc, const float* w,
                            const float* bias, int n_models, float* scores, hipStream_t s);
hipError_t launch_svm_wave(const float* blocks, const uint8_t* cells, int wc, int hc, const float* w,
                           const float* bias, int n_models, float* scores, hipStream_t s);

}  // namespace pd
