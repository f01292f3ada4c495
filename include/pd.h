/*
 * pd.h -- C ABI of libpd, the MI355X (gfx950) HOG+LBP+SVM pedestrian
 * detection hot path of Campmany et al., "GPU-based pedestrian detection for
 * autonomous driving" (arXiv 1611.01642).
 *
 * The pipeline, per frame (Section 4.1): build the scaled image pyramid,
 * extract HOG and LBP features on every level, score every sliding window
 * with linear SVMs, keep the windows above a threshold and refine them with
 * non-maximum suppression.
 *
 * Conventions shared by every entry point:
 *   - Every data pointer is a DEVICE pointer owned by the caller unless the
 *     argument says "host".  The library never allocates device memory on
 *     these calls; pd_detect takes a caller-provided workspace.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Every call only enqueues work on that stream and returns; results are
 *     visible after the caller synchronises the stream.
 *   - Images are 8-bit grayscale, row-major, with a row pitch in bytes
 *     (pitch >= width).
 *   - Return value: PD_OK or a negative PD_E_* code; pd_last_error() gives a
 *     message for the calling thread's last failure.  On an argument error
 *     nothing is enqueued.
 *   - Geometry is fixed: 8x8-pixel cells, 16x16-pixel blocks with a one-cell
 *     stride, 9 unsigned orientation bins, 59 uniform-LBP bins, 64x128
 *     windows anchored on the cell grid (stride 8 pixels).
 */
#ifndef PD_H
#define PD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PD_OK            0
#define PD_E_ARG        (-1)  /* null pointer, bad pitch, unknown flag       */
#define PD_E_SIZE       (-2)  /* non-positive or over-limit dimensions       */
#define PD_E_WORKSPACE  (-3)  /* workspace missing or too small              */
#define PD_E_HIP        (-4)  /* a HIP launch or copy reported an error      */
#define PD_E_OVERFLOW   (-5)  /* results complete but truncated: more
                                 candidates or kept boxes than capacity (the
                                 highest-scoring were kept, the true counts
                                 reported); returned only by calls that wait
                                 for their results (pd_video_pop)            */
#define PD_E_IO         (-6)  /* a file could not be read or written, or is
                                 not of the expected kind                    */

/* ---- fixed geometry ---------------------------------------------------- */
#define PD_CELL          8
#define PD_WIN_W         64
#define PD_WIN_H         128
#define PD_HOG_BINS      9
#define PD_HOG_BLOCK     36     /* 2x2 cells x 9 bins per block            */
#define PD_LBP_BINS      59
#define PD_WIN_BLOCKS_Y  15     /* HOG blocks per window: 15 x 7           */
#define PD_WIN_BLOCKS_X  7
#define PD_WIN_CELLS_Y   16     /* LBP cells per window: 16 x 8            */
#define PD_WIN_CELLS_X   8
#define PD_HOG_DIM       3780   /* 15 * 7 * 36                             */
#define PD_LBP_DIM       7552   /* 16 * 8 * 59                             */
#define PD_FEATURE_DIM   11332  /* PD_HOG_DIM + PD_LBP_DIM                 */
#define PD_LBP_BLOCK_DIM 6195   /* 15 * 7 * 59: LBP block histograms of a
                                   window (Algorithm 3)                     */
#define PD_BLOCK_MODEL_DIM 9975 /* PD_HOG_DIM + PD_LBP_BLOCK_DIM          */
#define PD_MAX_LEVELS    64
#define PD_MAX_DIM       16384  /* largest accepted image side             */
#define PD_MAX_MODELS    16
#define PD_MAX_CANDIDATES 4096  /* candidates per frame that NMS takes: the
                                   highest-scoring ones when a frame has more */

/* feature subsets (Section 4.1: LBP-SVM, HOG-SVM, HOGLBP-SVM) */
#define PD_FEAT_HOG      1
#define PD_FEAT_LBP      2

/* scoring precision */
#define PD_PREC_F32      0    /* FP32 features, FP32 scoring                  */
#define PD_PREC_BF16     1    /* BF16 HOG, BF16 MFMA scoring (FP32 sums) with
                                 FP64 rescoring of near-threshold windows     */
#define PD_MAX_MODELS_BF16 8  /* 8 models x {hi, lo} weight halves = 16 MFMA
                                 columns                                      */

/* ---- parameters -------------------------------------------------------- */
typedef struct pd_params {
    int32_t scale_num;   /* pyramid step as the ratio scale_num/scale_den,  */
    int32_t scale_den;   /*   e.g. 11/10; must satisfy num > den > 0         */
    int32_t max_levels;  /* 0: every level the 64x128 window fits in        */
    float   clip;        /* L2-Hys clip level (0.2)                         */
    float   eps;         /* L2-Hys epsilon (1e-3)                           */
    int32_t features;    /* PD_FEAT_HOG | PD_FEAT_LBP                       */
    int32_t precision;   /* PD_PREC_F32 or PD_PREC_BF16                     */
    float   margin;      /* PD_PREC_BF16: windows whose score is within
                            margin of the threshold are rescored in FP64
                            (0.05)                                          */
    /* Tile and launch shapes of pd_detect (0 = default).  They change the
       work partition only, never a result; pd_autotune picks them.        */
    int32_t tune_feat_rows;  /* block rows per feature strip: 4..32 (8)    */
    int32_t tune_score_rows; /* PD_PREC_F32 window rows per scoring band:
                                4, 8 or 16 (8)                             */
    int32_t tune_grid;       /* 0: default grids; n > 0: feature and
                                scoring grids of at most n workgroups
                                looping over the tiles                     */
    /* Learned window pruning (pd_detect; see the pruner section below):
       with prune_keep = K > 0 the network `pruner` (device float
       [PD_PRUNER_PARAMS]) runs on every level (BF16 MFMA) and, per frame,
       only windows whose logit is >= the K-th largest window logit of the
       frame (ties kept) can be detections; score tiles holding none of them
       are not scored.  0 = off (pruner ignored).                          */
    int32_t prune_keep;
    const float* pruner;
} pd_params;

/* Fills the defaults above: 11/10, all levels, 0.2, 1e-3, HOG|LBP, FP32,
   margin 0.05, default tile shapes, no pruning. */
void pd_params_default(pd_params* p);

/* One pyramid level as planned by pd_plan_pyramid (host struct). */
typedef struct pd_level {
    int32_t w, h;          /* level size in pixels                          */
    int32_t pitch;         /* row pitch in bytes inside the packed pyramid  */
    int32_t cells_x;       /* Wc = w / 8                                    */
    int32_t cells_y;       /* Hc = h / 8                                    */
    int32_t blocks_x;      /* Wb = Wc - 1                                   */
    int32_t blocks_y;      /* Hb = Hc - 1                                   */
    int32_t win_x;         /* window anchors per row: Wc - 7                */
    int32_t win_y;         /* window anchor rows:     Hc - 15               */
    int32_t reserved;
    int64_t offset;        /* byte offset of the level in the pyramid       */
} pd_level;

/*
 * pd_plan_pyramid -- host only, no GPU work.
 * Level k has size floor(w * den^k / num^k) x floor(h * den^k / num^k)
 * (Section 4.4, pyramidal sliding window; level 0 is the input itself);
 * levels are kept while the 64x128 window fits, up to params->max_levels.
 * Levels are packed one after another, each at a 256-byte aligned offset
 * with a pitch rounded up to 16 bytes.
 *   levels  : host array of `cap` entries, filled with the first
 *             min(n, cap) levels
 *   n_levels: host, receives n (0 when the image is smaller than a window:
 *             not an error)
 *   bytes   : host, receives the size of the packed pyramid buffer
 * Errors: PD_E_ARG (null params/outputs, bad scale), PD_E_SIZE (w or h
 * outside [1, PD_MAX_DIM]).
 */
int pd_plan_pyramid(int w, int h, const pd_params* params, pd_level* levels,
                    int cap, int* n_levels, int64_t* bytes);

/*
 * pd_build_pyramid -- Section 4.1 step (2), Section 4.4.
 * Writes every planned level into `pyr` (packed as planned) in one launch.
 * Level k is resampled from the level-0 image: output pixel (x, y) samples
 * the source at ((x + 0.5) w0 / wk - 0.5, (y + 0.5) h0 / hk - 0.5) in Q8
 * fixed point, bilinear, rounded half up; level 0 is an exact copy.
 *   img     : device, h rows of `pitch` bytes
 *   levels  : host array of n entries from pd_plan_pyramid
 *   pyr     : device, at least the `bytes` pd_plan_pyramid returned
 */
int pd_build_pyramid(const uint8_t* img, int w, int h, int pitch,
                     const pd_level* levels, int n, uint8_t* pyr, void* stream);

/*
 * pd_lbp_codes -- Section 4.2, Algorithm 1.
 * 8-bit LBP code of every pixel: neighbour k (TL,T,TR,R,BR,B,BL,L for
 * k = 0..7) sets bit k when it is >= the centre; neighbours outside the
 * image are clamped to the edge.
 *   codes   : device [h][codes_pitch] bytes
 */
int pd_lbp_codes(const uint8_t* lvl, int w, int h, int pitch,
                 uint8_t* codes, int codes_pitch, void* stream);

/*
 * pd_lbp -- Section 4.2, Algorithms 1 and 2.
 * Uniform-LBP cell histograms: every pixel of the Hc x Wc whole 8x8 cells
 * adds one count to its cell's bin (58 uniform codes in ascending order,
 * then one bin for all other codes).
 *   cell_hist: device uint8 [59][Hc][Wc] (bin-major planes; counts 0..64)
 */
int pd_lbp(const uint8_t* lvl, int w, int h, int pitch, uint8_t* cell_hist,
           void* stream);

/*
 * pd_hog -- Section 4.3, Algorithms 4 and 5, plus L2-Hys block
 * normalisation.  Gradient dx = I[y][x-1] - I[y][x+1],
 * dy = I[y-1][x] - I[y+1][x] (edge-clamped); orientation folded to
 * [0, 180) degrees; 9 bins centred at 10 + 20k degrees with linear
 * interpolation; bilinear spatial weights towards the four cell centres of
 * each 16x16 block; then v/sqrt(|v|^2+eps^2), clip, renormalise.
 *   blocks  : device float [36][Hb][Wb]; entry (r*2+c)*9+bin of block
 *             (by, bx) is plane (r*2+c)*9+bin
 */
int pd_hog(const uint8_t* lvl, int w, int h, int pitch, const pd_params* params,
           float* blocks, void* stream);

/*
 * pd_features -- pd_hog and pd_lbp of one level in a single pass over the
 * pixels.  HOG goes to `blocks` (FP32) or to `blocks_bf16` (the same values
 * rounded to nearest-even BF16, uint16 bit patterns, same [36][Hb][Wb]
 * layout); at most one of the two may be non-NULL.  Outputs that are NULL
 * are not computed.
 */
int pd_features(const uint8_t* lvl, int w, int h, int pitch, const pd_params* params,
                float* blocks, uint16_t* blocks_bf16, uint8_t* cell_hist, void* stream);

/*
 * pd_lbp_blocks -- Section 4.2, Algorithm 3 (the histogram reduction).
 * The 59-bin histogram of each 16x16-pixel block (blocks overlap by one
 * cell) as the sum of its four 8x8 cell histograms, for n images at once.
 *   cells   : device uint8 [n][59][hc][wc] (pd_lbp layout per image)
 *   blocks  : device uint16 [n][59][hc-1][wc-1] (a block counts 256 pixels)
 * Errors: PD_E_SIZE unless n >= 1, hc, wc >= 2 and the sides are within
 * PD_MAX_DIM / 8; PD_E_ARG on a NULL pointer.
 */
int pd_lbp_blocks(const uint8_t* cells, int n, int hc, int wc, uint16_t* blocks, void* stream);

/*
 * pd_fold_lbp_weights -- a linear model over HOG blocks and LBP block
 * histograms (Algorithm 3) as the cell-level model with the same window
 * scores.  Block-model layout per model: the 3780 HOG weights, then
 * [15][7][59] LBP block weights (window block row, column, bin).  Since a
 * block histogram is the plain sum of its four cells, the output's LBP weight
 * of window cell (a, b) is the sum of the weights of the window blocks
 * (a', b'), a' in {a-1, a}, b' in {b-1, b}, that contain it (FP32 sums in a
 * fixed order); HOG weights are copied.  pd_detect and pd_score_windows with
 * the folded weights then score with the block-level model.
 *   wb : device float [n_models][PD_BLOCK_MODEL_DIM]
 *   w  : device float [n_models][PD_FEATURE_DIM]
 * Errors: PD_E_SIZE when n_models is outside [1, PD_MAX_MODELS]; PD_E_ARG on
 * a NULL pointer.
 */
int pd_fold_lbp_weights(const float* wb, int n_models, float* w, void* stream);

/*
 * pd_score_windows -- Section 4.4, Algorithm 6.
 * For every window anchor (i, j), 0 <= i < Hc-15, 0 <= j < Wc-7:
 *   s_m(i,j) = sum_{a<15,b<7,c<36} blocks[c][i+a][j+b] * w_m[(a*7+b)*36+c]
 *            + sum_{a<16,b<8,c<59} cells[c][i+a][j+b] * w_m[3780+(a*8+b)*59+c]
 *            + bias_m
 * in FP32 (FP32 products and sums).
 *   blocks  : device float [36][Hc-1][Wc-1] (pd_hog layout)
 *   cells   : device uint8 [59][Hc][Wc] (pd_lbp layout)
 *   weights : device float [n_models][11332]
 *   bias    : device float [n_models]
 *   scores  : device float [n_models][Hc-15][Wc-7]
 * Errors: PD_E_SIZE when Hc < 16 or Wc < 8 or n_models outside
 * [1, PD_MAX_MODELS].
 */
int pd_score_windows(const float* blocks, const uint8_t* cells, int cells_x, int cells_y,
                     const float* weights, const float* bias, int n_models,
                     float* scores, void* stream);

/*
 * BF16 scoring (Section 4.4, Algorithm 6 as GEMMs on BF16 MFMA with FP32
 * accumulation).  LBP weights are carried as hi = bf16(w) plus lo =
 * bf16(w - hi) (LBP counts are exact); HOG weights as hi only (HOG features
 * are BF16).  One model: per feature row, a GEMM of windows x (b, c) x the
 * model's row offsets, then diagonal sums; 2..8 models: windows x features x
 * (models, hi/lo) for LBP and (models, two row offsets) for HOG, whose one
 * BF16 part per weight leaves room for a second window row.
 *
 * pd_packed_models_bytes -- bytes of the packed model buffer (any n_models).
 * pd_pack_models -- packs weights (device float [n_models][11332], layout of
 *   pd_score_windows, n_models <= PD_MAX_MODELS_BF16) into `packed` (device).
 * pd_score_windows_bf16 -- scores [n_models][Hc-15][Wc-7] (FP32) from BF16
 *   HOG planes [36][Hc-1][Wc-1] (uint16 bit patterns), uint8 LBP planes
 *   [59][Hc][Wc], packed models and bias (device float [n_models]).
 */
int64_t pd_packed_models_bytes(void);
int pd_pack_models(const float* weights, int n_models, uint16_t* packed, void* stream);
int pd_score_windows_bf16(const uint16_t* blocks_bf16, const uint8_t* cells, int cells_x, int cells_y,
                          const uint16_t* packed, const float* bias, int n_models, float* scores,
                          void* stream);

/* ---- the paper's own kernel mappings (ablation baselines) ------------------
 * The mappings the paper designs and measures (Section 4; px/ns comparisons
 * of Section 5.3), kept so that they can be timed beside this library's
 * kernels on the same GPU.  They compute the same results (up to FP32
 * rounding order); pd_detect does not use them.
 *
 * pd_lbp_naive -- Section 4.2, Naive scheme: a thread per 8x8 cell counts
 *   the cell's 64 codes of an LBP map (pd_lbp_codes output, [h][codes_pitch]
 *   bytes) in a private array.
 * pd_lbp_scatter -- Section 4.2, Scalable scheme (Algorithm 2): a thread per
 *   pixel adds 1 to its cell's bin with a global atomic (the histogram is
 *   cleared first).
 *   cell_hist: device uint32 [h/8][w/8][59] (the paper's cell-major layout;
 *   the uniform bins of pd_lbp).
 * pd_hog_global -- Section 4.3, Algorithms 4 and 5, the Global variant: a
 *   thread per pixel writes magnitude and orientation (degrees, [0, 180)) to
 *   grad (device float [2][h][w], caller-owned scratch); then a thread per
 *   16x16 block accumulates the block's trilinear histogram directly in
 *   `blocks` (global memory) and applies L2-Hys.  Same definition and layout
 *   as pd_hog: blocks float [36][Hb][Wb].
 * pd_score_windows_naive -- Section 4.4, Naive scheme: a thread per window.
 * pd_score_windows_wave -- Section 4.4, Algorithm 6 (warp-level): a wave per
 *   window, lanes striding over the 11332 features, shuffle-tree reduction.
 *   Both: the arguments, layouts and results of pd_score_windows.
 * Errors: PD_E_ARG on NULL pointers or a pitch below the width, PD_E_SIZE on
 * sizes outside the limits of the corresponding library call.
 */
int pd_lbp_naive(const uint8_t* codes, int w, int h, int codes_pitch, uint32_t* cell_hist, void* stream);
int pd_lbp_scatter(const uint8_t* codes, int w, int h, int codes_pitch, uint32_t* cell_hist, void* stream);
int pd_hog_global(const uint8_t* lvl, int w, int h, int pitch, const pd_params* params, float* grad,
                  float* blocks, void* stream);
int pd_score_windows_naive(const float* blocks, const uint8_t* cells, int cells_x, int cells_y,
                           const float* weights, const float* bias, int n_models, float* scores,
                           void* stream);
int pd_score_windows_wave(const float* blocks, const uint8_t* cells, int cells_x, int cells_y,
                          const float* weights, const float* bias, int n_models, float* scores,
                          void* stream);

/* ---- whole pipeline ------------------------------------------------------ */

/* One input frame (device image). */
typedef struct pd_frame {
    const uint8_t* data;
    int32_t w, h, pitch;
    int32_t reserved;
} pd_frame;

/* One detection, in original-image coordinates of its frame. */
typedef struct pd_box {
    int32_t frame, level, i, j, model;
    int32_t x0, y0, x1, y1;  /* box in 1/256 pixels: x0 = floor(256*8j*w0/wk),
                                x1 = floor(256*(8j+64)*w0/wk), y likewise
                                with 128 and the heights                    */
    float   score;           /* window score (max over models)             */
    double  score64;         /* FP64 rescore (PD_PREC_BF16, windows within
                                the margin of the threshold), else NaN     */
} pd_box;

/* Per-frame result counters written by pd_detect. */
typedef struct pd_counts {
    int32_t candidates;  /* windows with score > threshold (true count; every
                            one is in the frame's candidate list)          */
    int32_t kept;        /* boxes written after NMS (<= cap)               */
    int32_t overflow;    /* 1 if candidates > PD_MAX_CANDIDATES or the kept
                            boxes exceeded `cap`.  Past PD_MAX_CANDIDATES,
                            NMS runs on the PD_MAX_CANDIDATES highest-scoring
                            candidates (score descending, then level, i, j
                            ascending: a strict order, so the same inputs
                            always give the same boxes); past `cap`, the
                            first `cap` kept boxes (the highest-scoring)
                            are written                                    */
    int32_t rescored;    /* PD_PREC_BF16: windows rescored in FP64 (every
                            window within the margin of the threshold)     */
} pd_counts;

/*
 * pd_detect_workspace_bytes -- host only.  Size of the device workspace
 * pd_detect needs for these frame sizes (host array `frames`, only w and h
 * are read) and n_models.  Returns a negative PD_E_* code on bad input.
 */
int64_t pd_detect_workspace_bytes(const pd_frame* frames, int n_frames,
                                  const pd_params* params, int n_models);

/*
 * pd_detect -- the whole hot path for a batch of device-resident frames of
 * any sizes (Section 4.1 steps 2-5): pyramid, features, window scores,
 * threshold (a window is a detection iff its score, the max over models,
 * is > thresholds[frame]) and greedy NMS (order by score descending, then
 * level, i, j ascending).  With params->precision == PD_PREC_BF16 (at most
 * 8 models) the HOG features are stored in BF16, scores come from BF16 MFMA,
 * and every window whose score is within params->margin of the threshold is
 * recomputed from its pixels in FP64 (no matter how many: the near list has
 * room for every window of the batch); its FP64 score decides.  With a
 * feature subset (params->features), BF16 scoring and the FP64 rescore read
 * only that family's features and weights.  Every candidate (window above
 * the threshold) of a frame is kept in a list sized by the frame's window
 * count; NMS runs on at most PD_MAX_CANDIDATES of them, the highest-scoring
 * (see pd_counts).  A box is suppressed iff its IoU with a kept box is >
 * 0.5, decided exactly as 2*inter > union on the integer boxes.  Every stage
 * is one launch over all frames and levels.
 *   frames     : host array of n_frames descriptors (device images)
 *   weights    : device float [n_models][11332], bias: device [n_models]
 *   thresholds : device double [n_frames]
 *   workspace  : device, >= pd_detect_workspace_bytes(...) bytes
 *   boxes      : device pd_box [n_frames][cap], kept boxes in NMS order
 *   counts     : device pd_counts [n_frames]
 * Errors, found on the host before any GPU work: PD_E_ARG on bad params, a
 * NULL pointer, a frame pitch below its width, cap < 0, n_frames < 1 (an
 * empty batch is an error, not a no-op) or a workspace not 256-byte aligned; PD_E_SIZE when n_models is
 * outside [1, PD_MAX_MODELS] ([1, PD_MAX_MODELS_BF16] in BF16) or a frame's
 * sides are outside [1, PD_MAX_DIM]; PD_E_WORKSPACE when workspace_bytes is
 * below pd_detect_workspace_bytes.
 */
int pd_detect(const pd_frame* frames, int n_frames, const float* weights,
              const float* bias, int n_models, const pd_params* params,
              const double* thresholds, void* workspace, int64_t workspace_bytes,
              pd_box* boxes, int cap, pd_counts* counts, void* stream);

/*
 * pd_detect_noalloc -- pd_detect for callers that cannot allocate memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as pd_detect, but no
 * workspace: it uses a static device array of PD_NOALLOC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends, and it
 * passes its tables to the device as kernel arguments, so it calls no
 * hipMalloc, hipFree, hipHostMalloc or other device or pinned allocator.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (on different streams, or from different threads) race.  Consecutive calls
 * on one stream are safe: each clears its counters before use.
 * Errors: those of pd_detect; PD_E_WORKSPACE, before any GPU work, when the
 * batch needs more than PD_NOALLOC_SCRATCH_BYTES of workspace
 * (pd_detect_workspace_bytes: a 1242x375 frame needs about 10 MiB, a
 * 1920x1080 frame about 50 MiB).
 */
#define PD_NOALLOC_SCRATCH_BYTES (64ll << 20)
int pd_detect_noalloc(const pd_frame* frames, int n_frames, const float* weights,
                      const float* bias, int n_models, const pd_params* params,
                      const double* thresholds, pd_box* boxes, int cap,
                      pd_counts* counts, void* stream);

/*
 * pd_graph_create -- the kernel sequence of pd_detect on exactly these
 * arguments, captured once into a HIP graph for replay by pd_graph_launch
 * (HIP graph capture in place of per-call launches; the work is that of
 * Section 4.1 steps 2-5 as in pd_detect).  The call allocates device memory
 * for the graph's own copy of the level and tile tables (freed by
 * pd_graph_destroy), uploads them now and waits for that copy on `stream`;
 * the graph holds kernels only (the counters are cleared by a kernel).  So
 * pd_detect, pd_autotune or other graphs may use the same workspace between
 * launches (one at a time: they share its feature and candidate buffers).
 * Every pointer argument is baked into the graph: the frames, weights, bias,
 * thresholds, workspace, boxes and counts must stay allocated until
 * pd_graph_destroy, and their contents may change between launches (new
 * pixels in the same frame buffers, new thresholds or weights).  Frame sizes
 * and params are fixed.  Launches of one graph must not overlap (they share
 * the workspace).
 *   out : host pointer receiving the graph handle
 * Errors: those of pd_detect; PD_E_HIP if capture or instantiation fails.
 */
typedef struct pd_graph pd_graph;
int pd_graph_create(const pd_frame* frames, int n_frames, const float* weights,
                    const float* bias, int n_models, const pd_params* params,
                    const double* thresholds, void* workspace, int64_t workspace_bytes,
                    pd_box* boxes, int cap, pd_counts* counts, void* stream,
                    pd_graph** out);

/* pd_graph_launch -- enqueue one replay of the captured pipeline on stream. */
int pd_graph_launch(pd_graph* graph, void* stream);

/* pd_graph_destroy -- release the graph (NULL is accepted); the caller makes
   sure no launch is still running. */
int pd_graph_destroy(pd_graph* graph);

/* ---- detection context: tuning table and graph cache ---------------------- */
/*
 * A context keeps, across calls:
 *   - a tuning table: the tile and grid shapes chosen for a batch shape (the
 *     sequence of frame sizes, n_models, and the params that shape the work:
 *     scale, max_levels, features, precision, pruning on/off), filled by
 *     pd_ctx_autotune or pd_ctx_set_tuning, saved and loaded as text;
 *   - a graph cache: pd_ctx_detect captures a call's kernel sequence once
 *     (as pd_graph_create) and replays it for every later call with the same
 *     arguments (same buffers, sizes and params; buffer contents may change),
 *     so repeated calls skip the host's table build and upload.  At most 8
 *     graphs are kept; the least recently used is released once its last
 *     launch has finished.
 * A context is used by one thread at a time.  pd_ctx_create and
 * pd_ctx_detect allocate host memory, and the first pd_ctx_detect on a new
 * set of arguments allocates the graph's table memory and waits for its
 * upload (as pd_graph_create); later calls on those arguments allocate
 * nothing.
 */
typedef struct pd_ctx pd_ctx;
int pd_ctx_create(pd_ctx** out);
/* Waits for the cached graphs' last launches, then releases everything. */
int pd_ctx_destroy(pd_ctx* ctx);
/*
 * pd_ctx_detect -- pd_detect (Section 4.1 steps 2-5) through the context:
 * when params leave every tuning field at 0 and the table has an entry for
 * this batch shape, that entry's fields are used; the call is then replayed
 * from the graph cache (captured first if these arguments are new).  With
 * pd_profile_enable on, it runs as an eager pd_detect (stage events).
 * Arguments, results and errors: those of pd_detect and pd_graph_create.
 */
int pd_ctx_detect(pd_ctx* ctx, const pd_frame* frames, int n_frames, const float* weights,
                  const float* bias, int n_models, const pd_params* params,
                  const double* thresholds, void* workspace, int64_t workspace_bytes,
                  pd_box* boxes, int cap, pd_counts* counts, void* stream);
/*
 * pd_ctx_autotune -- pd_autotune, remembered: when the table already holds
 * this batch shape, *best is params with its fields (and *best_ms the time
 * stored with them) and nothing runs; otherwise pd_autotune runs and its
 * choice is stored.  Arguments and errors: those of pd_autotune.
 */
int pd_ctx_autotune(pd_ctx* ctx, const pd_frame* frames, int n_frames, const float* weights,
                    const float* bias, int n_models, const pd_params* params,
                    const double* thresholds, void* workspace, int64_t workspace_bytes,
                    pd_box* boxes, int cap, pd_counts* counts, int iters, pd_params* best,
                    float* best_ms, void* stream);
/*
 * pd_ctx_tuning -- host only: *out = params with the table's tuning fields
 * for this batch shape.  Returns 1 if the table had an entry, 0 if not (then
 * *out = params), or a negative PD_E_* code (frames, params or n_models
 * invalid, as for pd_detect_workspace_bytes).  Only w and h of the frames are
 * read.
 */
int pd_ctx_tuning(const pd_ctx* ctx, const pd_frame* frames, int n_frames, const pd_params* params,
                  int n_models, pd_params* out);
/* pd_ctx_set_tuning -- host only: stores params' tuning fields (and `ms`)
   as the entry of this batch shape.  Errors as pd_ctx_tuning. */
int pd_ctx_set_tuning(pd_ctx* ctx, const pd_frame* frames, int n_frames, const pd_params* params,
                      int n_models, float ms);
/*
 * pd_ctx_save / pd_ctx_load -- the tuning table as a text file: a first
 * line "pd-tuning 1", then one line per entry, "<shape>\t<feat_rows>
 * <score_rows> <grid> <ms>".  Loading adds the file's entries (replacing
 * those with the same shape) only if the whole file is valid.
 * Errors: PD_E_IO when the file cannot be opened, read or written, or a line
 * is malformed or out of range; PD_E_ARG on NULL arguments.
 */
int pd_ctx_save(const pd_ctx* ctx, const char* path);
int pd_ctx_load(pd_ctx* ctx, const char* path);

/*
 * pd_graph_stage_ms -- for a graph created while pd_profile_enable was on
 * (the capture then holds, before each stage and after the last one, a
 * one-wave kernel that writes the device's constant-rate clock into a slot
 * the graph owns): waits for the device to go idle and writes to host
 * ms[PD_N_STAGES] the most recent launch's time per stage (the upload stage
 * is ~0: a graph holds no copy).  Before the first launch the values are
 * meaningless.
 * Errors: PD_E_ARG if graph is NULL or was captured without stage stamps;
 * PD_E_HIP from the device queries.
 */
int pd_graph_stage_ms(pd_graph* graph, double* ms);

/* ---- streaming video (Section 4.1 steps 1 and 5 around steps 2-4) ------- */
/*
 * A video stream of frames of one size that arrive one at a time in host
 * memory.  Each push copies the frame to the GPU (step 1), runs pd_detect's
 * kernels on it (steps 2-4 and NMS, as a graph captured at creation) and
 * copies the counts and boxes back (step 5), on three streams ordered by
 * events, so the copies of one frame overlap the detection of its
 * neighbours.  Up to `depth` frames are in flight; results come back in push
 * order.  This object owns its buffers: pd_video_create allocates device
 * memory (frames, workspaces, results) and pinned host memory for `depth`
 * slots, and pd_video_destroy frees them; push and pop allocate nothing.
 * One video must not be used from two threads at once.
 */
#define PD_VIDEO_MAX_DEPTH 16
typedef struct pd_video pd_video;

/*
 * pd_video_create -- frames of w x h pixels, detected with `params` (tuning
 * fields included) and the models (device weights [n_models][11332], bias
 * [n_models], kept alive by the caller until pd_video_destroy); up to `cap`
 * boxes per frame; `depth` in [1, PD_VIDEO_MAX_DEPTH] frames in flight.
 * Blocks until the set-up finished.
 *   out : host pointer receiving the handle
 * Errors: those of pd_detect_workspace_bytes; PD_E_SIZE for depth, cap or the
 * frame size; PD_E_HIP when an allocation or the capture fails.
 */
int pd_video_create(int w, int h, const pd_params* params, const float* weights,
                    const float* bias, int n_models, int cap, int depth, pd_video** out);

/*
 * pd_video_push -- queue one frame (host memory, `pitch` bytes per row,
 * copied before the call returns) with its detection threshold.  Returns
 * without waiting for the GPU.
 * Errors: PD_E_SIZE when `depth` frames are already in flight (pop first);
 * PD_E_ARG on a NULL frame or pitch < w.
 */
int pd_video_push(pd_video* v, const uint8_t* frame, int pitch, double threshold);

/*
 * pd_video_pop -- wait for the oldest frame in flight and copy its counts and
 * up to `cap` boxes (host buffers, NMS order, frame index 0) to the caller.
 * `device_ms` (host, may be NULL) receives the GPU time from the start of its
 * upload to the end of its download, queueing behind earlier frames included.
 * Errors: PD_E_ARG when no frame is in flight or on a NULL pointer;
 * PD_E_OVERFLOW (the frame is popped and its counts and boxes written) when
 * its counts report an overflow or it kept more boxes than `cap`.
 */
int pd_video_pop(pd_video* v, pd_box* boxes, int cap, pd_counts* counts, float* device_ms);

/* pd_video_destroy -- wait for work in flight and free the video's buffers
   (NULL is accepted). */
int pd_video_destroy(pd_video* v);

/*
 * pd_autotune -- times pd_detect's kernel sequence on these arguments, as
 * captured graphs (the device's time, without the host's table build and
 * upload), over the tuning fields of pd_params: per candidate, against the
 * current choice, three rounds of (capture, one untimed launch, `iters`
 * launches between HIP events) for each in turn, the least time of each
 * compared.  Fields tried one at a time: feature strip rows {4, 6, 8, 10,
 * 12, 14, 16}, FP32 scoring rows {4, 8, 16}, grid cap {0, 256, 512, 1024,
 * 2048};
 * starting from params' own values.  Writes params with the fastest fields to
 * *best (host) and its device time per call in ms to *best_ms (host, may be
 * NULL).  Blocks until the timing runs finished; leaves boxes and counts of
 * the last run.  The workspace size does not depend on the tuning fields;
 * the next pd_detect call uploads its own tables as always.
 * Errors: those of pd_detect; PD_E_ARG for iters outside [1, 1000].
 */
int pd_autotune(const pd_frame* frames, int n_frames, const float* weights,
                const float* bias, int n_models, const pd_params* params,
                const double* thresholds, void* workspace, int64_t workspace_bytes,
                pd_box* boxes, int cap, pd_counts* counts, int iters,
                pd_params* best, float* best_ms, void* stream);

/* ---- learned window pruner ------------------------------------------------
 * Not part of the paper: a small network over per-cell features predicts
 * which windows the linear SVM (Section 4.4) will score above the threshold,
 * so that the others need not be scored.
 *   cell map  : per 8x8 cell, 68 FP32 channels, planar [68][cells_y][cells_x]:
 *               the cell's 9-bin orientation histogram (Section 4.3, the
 *               gradients of Algorithm 4 and the votes of Algorithm 5) with
 *               the full bilinear spatial kernel -- every pixel whose centre
 *               is within 8 px per axis of the cell centre votes with weight
 *               (1 - |dy|/8)(1 - |dx|/8) -- divided by sqrt(|h|^2 + eps^2),
 *               then the 59 uniform-LBP counts (Section 4.2) / 64.
 *   network   : conv3x3 68->32, ReLU, conv3x3 32->32, ReLU, conv3x3 32->16,
 *               ReLU, 1x1 16->1; zero padding; one logit per cell; window
 *               (i, j) takes the logit of cell (i + 7, j + 3).
 *   parameters: one float vector of PD_PRUNER_PARAMS values: per conv layer
 *               weights [Cout][Cin][3][3] then bias [Cout]; then the head's
 *               weights [16] and bias [1].
 */
#define PD_PRUNER_CHANNELS 68
#define PD_PRUNER_PARAMS   33505

/* One map (pyramid level) of a pruner call; every pointer is a device
   pointer, planar FP32, owned by the caller. */
typedef struct pd_net_map {
    const float* cellmap;  /* [68][cells_y][cells_x]                          */
    float* logits;         /* [cells_y][cells_x], written                     */
    const float* labels;   /* [cells_y][cells_x] 0/1, pd_pruner_gradient only */
    const float* mask;     /* [cells_y][cells_x] 0/1, pd_pruner_gradient only */
    int32_t cells_x, cells_y;
} pd_net_map;

/*
 * pd_features_cellmap -- pd_features (FP32 HOG blocks and LBP cell counts)
 * and, from the same pass over the pixels, the pruner's cell map of the
 * level.  blocks [36][Hb][Wb], cell_hist [59][Hc][Wc] u8, cellmap
 * [68][Hc][Wc] FP32 (device, caller-owned).  The HOG normalisation's eps
 * (params->eps) is also the cell map's.  Errors: PD_E_SIZE if the level has
 * no 16x16 block.
 */
int pd_features_cellmap(const uint8_t* level, int w, int h, int pitch, const pd_params* params,
                        float* blocks, uint8_t* cell_hist, float* cellmap, void* stream);

/* Workspace (device bytes, 256-byte aligned) of pd_pruner_forward and
   pd_pruner_gradient for these maps (host array; sizes only are read). */
int64_t pd_pruner_workspace_bytes(const pd_net_map* maps, int n_maps);

/* pd_pruner_forward -- logits of every map (FP32 throughout). */
int pd_pruner_forward(const pd_net_map* maps, int n_maps, const float* params,
                      void* workspace, int64_t workspace_bytes, void* stream);

/*
 * pd_pruner_gradient -- forward, then the gradient of the class-weighted
 * binary cross-entropy L = (1/N) sum over masked cells of
 * -pos_weight*y*log(s) - (1 - y)*log(1 - s), s = sigmoid(logit), N = number
 * of masked cells over all maps.  grad: device float [PD_PRUNER_PARAMS]
 * (layout of params); stats: device double [2] = (L, N).  Deterministic:
 * the same inputs give the same bits.
 */
int pd_pruner_gradient(const pd_net_map* maps, int n_maps, const float* params, float pos_weight,
                       float* grad, double* stats, void* workspace, int64_t workspace_bytes,
                       void* stream);

/*
 * pd_adam_step -- one Adam update (Kingma and Ba, bias-corrected) of n
 * FP32 parameters in place: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * step >= 1 counts updates.  All arrays are device float [n].
 */
int pd_adam_step(float* params, const float* grad, float* m, float* v, int n, int step, float lr,
                 float beta1, float beta2, float eps, void* stream);

/*
 * pd_window_labels -- training targets of one level: labels[cy][cx] = 1 iff
 * window (cy - 7, cx - 3) exists and its score (scores [win_y][win_x], e.g.
 * the max over models) is > *threshold (device double); mask = 1 where the
 * window exists.  Requires cells = windows + (7, 15) per axis.
 */
int pd_window_labels(const float* scores, int win_x, int win_y, int cells_x, int cells_y,
                     const double* threshold, float* labels, float* mask, void* stream);

/*
 * pd_pruner_save / pd_pruner_load -- training checkpoints of the pruner: its
 * parameters and Adam's first and second moments (device float
 * [PD_PRUNER_PARAMS] each), the number of Adam steps taken and the seed of
 * the training order, in a binary file `path` (host string): magic
 * "PDPRUNE1", version, parameter count, step, seed, the three vectors as
 * little-endian float32, an FNV-1a 64-bit checksum.  Save writes a sibling
 * file and renames it over `path`.  Both copy through host memory on
 * `stream` and synchronise it before returning.  Load may take NULL moment
 * pointers (inference only).
 * Errors: PD_E_ARG on NULL arguments or a negative step; PD_E_IO when the
 * file cannot be written or read, or is not a valid checkpoint (size, magic,
 * version, checksum); PD_E_HIP from the copies.
 */
int pd_pruner_save(const char* path, const float* params, const float* adam_m, const float* adam_v,
                   int64_t step, uint64_t seed, void* stream);
int pd_pruner_load(const char* path, float* params, float* adam_m, float* adam_v, int64_t* step,
                   uint64_t* seed, void* stream);

/*
 * pd_pruner_logits_bf16 -- the inference form of the pruner on one level
 * (w x h >= 64x128): features and the cell map in one pass (the cell map
 * stored channels-last in BF16), then the network on BF16 MFMA with FP32
 * accumulation (bias, ReLU and head in FP32; layer outputs rounded to
 * BF16).  logits: device float [h/8][w/8].  Workspace (device, 256-byte
 * aligned) from pd_pruner_logits_bf16_workspace_bytes(w, h).
 */
int64_t pd_pruner_logits_bf16_workspace_bytes(int w, int h);
int pd_pruner_logits_bf16(const uint8_t* level, int w, int h, int pitch, const pd_params* params,
                          const float* pruner, float* logits, void* workspace, int64_t workspace_bytes,
                          void* stream);

/*
 * pd_detect_candidates -- test hook: after pd_detect on the same arguments
 * (frames, params, n_models, workspace), enqueue copies of the first `cap`
 * entries of frame `frame`'s candidate list (windows above the threshold,
 * before NMS, in no particular order; the list holds
 * pd_counts.candidates entries, every candidate of the frame):
 *   cand_score : device float [cap]; cand_key: device int32 [cap][4] =
 *                (level, i, j, model); cand_s64: device double [cap] or NULL
 *                (FP64 score for rescored windows, NaN otherwise; PD_PREC_BF16)
 */
int pd_detect_candidates(const pd_frame* frames, int n_frames, const pd_params* params, int n_models,
                         const void* workspace, int64_t workspace_bytes, int frame, float* cand_score,
                         int32_t* cand_key, double* cand_s64, int cap, void* stream);
/* Errors: PD_E_SIZE when cap exceeds the frame's window count. */

/*
 * pd_nms -- greedy NMS of one candidate list (the last stage of pd_detect,
 * exposed for testing).  Candidates are windows of one frame:
 *   cand_score : device float [n]; cand_key: device int32 [n][4] =
 *                (level, i, j, model)
 *   level_wh   : host int32 [n_levels][2] level sizes, (w0, h0) = level 0
 *   boxes      : device pd_box [cap]; counts: device pd_counts [1]
 * Keys name levels in [0, n_levels) and anchors below 2048 (an out-of-range
 * level is clamped).  Errors: PD_E_SIZE when n > PD_MAX_CANDIDATES.
 */
int pd_nms(const float* cand_score, const int32_t* cand_key, int n,
           const int32_t* level_wh, int n_levels, pd_box* boxes, int cap,
           pd_counts* counts, void* stream);

/* ---- stage timing ---------------------------------------------------------- */
/* Stages of pd_detect, in launch order. */
#define PD_STAGE_UPLOAD   0   /* host tables -> workspace copy              */
#define PD_STAGE_ZERO     1   /* candidate counters cleared                 */
#define PD_STAGE_RESIZE   2   /* pyramid levels 1..n of every frame         */
#define PD_STAGE_FEATURES 3   /* HOG + LBP of every level                   */
#define PD_STAGE_SCORE    4   /* window scores of every level and model     */
#define PD_STAGE_COMPACT  5   /* threshold + candidate lists                */
#define PD_STAGE_NMS      6   /* greedy NMS per frame                       */
#define PD_N_STAGES       7

/*
 * pd_profile_enable -- when on != 0, every later pd_detect call on this host
 * thread records a HIP event on its stream before each stage and after the
 * last one (the only cost is the event records).  on == 0 stops recording.
 */
int pd_profile_enable(int on);

/*
 * pd_profile_read -- waits for the recorded events, then writes to host
 * ms[PD_N_STAGES] the summed GPU time of each stage over the recorded calls
 * and to *calls their number; reset != 0 clears the record afterwards.
 */
int pd_profile_read(double* ms, int64_t* calls, int reset);

/* ---- diagnostics ----------------------------------------------------------- */
const char* pd_strerror(int code);
const char* pd_last_error(void);   /* calling thread's last failure message */
const char* pd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PD_H */
