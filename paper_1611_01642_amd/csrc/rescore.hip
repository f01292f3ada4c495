// FP64 rescoring of near-threshold windows.
//
// After BF16 scoring, a window whose score lies within `margin` of its
// frame's threshold cannot be classified safely (Section 4.4: positive iff
// the distance to the hyper-plane exceeds the threshold).  This kernel
// recomputes such a window's features from the pixels of its pyramid level in
// FP64 -- gradients (Algorithm 4; orientation and magnitude from a table of
// every integer gradient, built in FP64 with the device's double atan2), trilinear
// HOG votes (Algorithm 5) as per-cell direction partials, L2-Hys -- takes its
// LBP counts (exact integers) from the feature planes, and scores every model
// in FP64 with the FP32 weights.  A window whose FP64 score (max over models)
// exceeds the threshold is appended to the frame's candidate list.
//
// One workgroup per near window, in two passes over the window's cell rows
// (rows 0..7, then 8..15), so that the FP64 partials of 9 cell rows at a time
// fit in LDS beside the pixels and two workgroups share a CU:
//  * pixels: the window's 130 x 66 pixels (with halo) in LDS;
//  * votes: in a pass, the four lanes l, l + 16, l + 32, l + 48 of a wave own
//    one of the pass's 64 cells, two pixel rows each; a lane sums its 16
//    pixels' votes in registers (the linear orientation vote as a hat over
//    the 9 bins, towards the 2 x 3 target cells its rows can reach), the four
//    quarters meet through cross-lane exchanges in a fixed order and the
//    cell's 81 direction partials are stored once (no read-modify-write in
//    LDS), in a ring of 9 cell rows (row r at r % 9);
//  * blocks: pass 1 builds block rows 0..6 (cell rows 0..7), pass 2 block rows
//    7..14 (cell rows 7..15: row 7 is still in the ring); a lane per block
//    sums the partials aimed at each slot (exactly Algorithm 5's votes),
//    L2-Hys, and stores the block's 36 HOG values;
//  * dot products: after each pass's blocks, all 256 lanes stride over its
//    HOG values (and after pass 2 over the LBP counts, staged over the
//    pixels) with coalesced FP32 weights (one model: 16 features in flight
//    per lane; several: four consecutive features per lane and step, one
//    16-byte weight load per model, 8 x 8 in flight), then a fixed-order
//    reduction;
//  * gathers: a thread issues all of its pixel (and LBP count) loads before
//    it stores any of them in LDS, so each gather costs one memory latency;
//    pixel rows and LBP runs are read as aligned 4-byte words where the
//    window allows it.
#include "pd_internal.h"

namespace pd {
namespace {

constexpr int RS_PY = PD_WIN_H + 2;  // 130 pixel rows incl. halo
constexpr int RS_PX = PD_WIN_W + 2;  // 66 pixel columns incl. halo
constexpr int RS_CELLS = PD_WIN_CELLS_Y * PD_WIN_CELLS_X;  // 128

// LDS pixel rows: byte RS_PX0 + c holds window column c - 1 (c = 0 .. 65),
// so that a row's source bytes from an aligned word boundary land on aligned
// LDS words
constexpr int RS_PX0 = 3;
constexpr int RS_ROW = 72;                 // 18 words per row
constexpr int RS_ROW_WORDS = RS_ROW / 4;

constexpr int RS_RING = 9;                                        // cell rows of partials in LDS
constexpr int RS_BLK1 = (PD_WIN_CELLS_Y / 2 - 1) * PD_WIN_BLOCKS_X;  // pass 1: block rows 0..6 (49 blocks)
constexpr int RS_BLK2 = PD_WIN_BLOCKS_Y * PD_WIN_BLOCKS_X - RS_BLK1;  // pass 2: block rows 7..14 (56)
constexpr int RS_HOG1 = RS_BLK1 * PD_HOG_BLOCK;                    // HOG features of pass 1 (1764)

struct RescoreShared {
    union {
        uint8_t px[RS_PY][RS_ROW];   // the window's pixels (votes)
        uint8_t lbp[PD_LBP_DIM];     // then its LBP counts, feature order (cell, bin)
    } p;
    double A[RS_RING * PD_WIN_CELLS_X][81];  // per cell: 3x3 target cells x 9 bins
    double hog[RS_BLK2 * PD_HOG_BLOCK];      // one pass's normalised HOG values
    double part[2][4][8];                    // per pass, wave, model
};

constexpr int RS_PX_PER_T = (RS_PY * RS_PX + 255) / 256;   // pixel bytes gathered per thread (border windows)
constexpr int RS_PXW_PER_T = (RS_PY * RS_ROW_WORDS + 255) / 256;  // pixel words per thread (inner windows)
constexpr int RS_LBP_RUNS = PD_LBP_BINS * PD_WIN_CELLS_Y;  // 8-byte runs: one plane row of the window
constexpr int RS_RUNS_PER_T = (RS_LBP_RUNS + 255) / 256;

// Per-model partial dot products of the window's features (LDS) with the
// weights over features [k_begin, k_end) (the whole vector, or one feature
// family), M = 1 or 8 models unrolled (models past n_models repeat the last
// one; their sums are never read).  Thread t takes features k_begin + t +
// 256 u; U features per step, so a thread's M * U weight loads are in flight
// together.  Past k_end x is 0 and the weight index is clamped.
template <int M>
__device__ __forceinline__ void dot_models(RescoreShared& sm, const float* __restrict__ weights, int n_models,
                                           int k_begin, int k_end, int hog_base, int pass, int t, int wave,
                                           int lane) {
    constexpr int U = M == 1 ? 16 : 3;
    double part[M];
#pragma unroll
    for (int m = 0; m < M; ++m) part[m] = 0.0;
    for (int k0 = k_begin + t; k0 < k_end; k0 += 256 * U) {
        float w[U][M];
        double x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + 256 * u;
            const int kc = min(k, k_end - 1);
#pragma unroll
            for (int m = 0; m < M; ++m) w[u][m] = weights[(size_t)min(m, n_models - 1) * PD_FEATURE_DIM + kc];
            const double xv = kc < PD_HOG_DIM ? sm.hog[kc - hog_base] : (double)sm.p.lbp[kc - PD_HOG_DIM];
            x[u] = k < k_end ? xv : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int m = 0; m < M; ++m) part[m] = fma(x[u], (double)w[u][m], part[m]);
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        double s = part[m];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) sm.part[pass][wave][m] = s;
    }
}

// The same with each thread taking four consecutive features per step
// (groups g = g_begin + t + 256 u of 4: one 16-byte weight load per model;
// 1764, 3780 and 11332 are multiples of 4, so a group is all HOG or all LBP
// and lies in one pass).
// Needs 16-byte aligned weights.
template <int M>
__device__ __forceinline__ void dot_models4(RescoreShared& sm, const float4* __restrict__ w4, int n_models,
                                            int g_begin, int g_end, int hog_base, int pass, int t, int wave,
                                            int lane) {
    constexpr int G = PD_FEATURE_DIM / 4;
    constexpr int U = M == 1 ? 4 : 1;
    double part[M];
#pragma unroll
    for (int m = 0; m < M; ++m) part[m] = 0.0;
    for (int g0 = g_begin + t; g0 < g_end; g0 += 256 * U) {
        float4 w[U][M];
        double x[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int g = g0 + 256 * u;
            const int gc = min(g, g_end - 1);
#pragma unroll
            for (int m = 0; m < M; ++m) w[u][m] = w4[(size_t)min(m, n_models - 1) * G + gc];
            const int k = 4 * gc;
            if (k < PD_HOG_DIM) {
#pragma unroll
                for (int j = 0; j < 4; ++j) x[u][j] = sm.hog[k - hog_base + j];
            } else {
                const uint32_t b = *reinterpret_cast<const uint32_t*>(&sm.p.lbp[k - PD_HOG_DIM]);
#pragma unroll
                for (int j = 0; j < 4; ++j) x[u][j] = (double)((b >> (8 * j)) & 255u);
            }
            if (g >= g_end) {
#pragma unroll
                for (int j = 0; j < 4; ++j) x[u][j] = 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int m = 0; m < M; ++m) {
                part[m] = fma(x[u][0], (double)w[u][m].x, part[m]);
                part[m] = fma(x[u][1], (double)w[u][m].y, part[m]);
                part[m] = fma(x[u][2], (double)w[u][m].z, part[m]);
                part[m] = fma(x[u][3], (double)w[u][m].w, part[m]);
            }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        double s = part[m];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) sm.part[pass][wave][m] = s;
    }
}

// The gradient table: for dy in 0..255 and dx in -255..255, the
// orientation's bin coordinate t = angle / 20 - 0.5 in [-0.5, 8.5) (angle in
// degrees, folded into [0, 180): Algorithm 4 with the device's double atan2)
// and the magnitude sqrt(dx^2 + dy^2), both FP64.  A gradient with dy < 0
// looks up (-dx, -dy): the same magnitude and, mathematically, the same
// folded angle (its FP64 value may differ in the last bits).
__global__ void orient_table_kernel(double2* __restrict__ table) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ORIENT_W * ORIENT_H) return;
    const int dy = e / ORIENT_W, dx = e - dy * ORIENT_W - 255;
    const double mag = sqrt((double)(dx * dx + dy * dy));
    double ang = atan2((double)dy, (double)dx) * 57.295779513082320876798154814105;
    if (ang < 0.0) ang += 180.0;
    if (ang >= 180.0) ang -= 180.0;
    table[e] = make_double2(ang / 20.0 - 0.5, mag);
}

// Bilinear weight of pixel offset p in [0, 8) of a cell towards cell d in {-1, 0, 1}.
__device__ __forceinline__ double spatial_w(int p, int d) {
    const double w = 1.0 - fabs((double)p + 0.5 - (8.0 * d + 4.0)) / 8.0;
    return w > 0.0 ? w : 0.0;
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) rescore64_kernel(const LevelItem* __restrict__ items,
                                                        const int32_t* __restrict__ first_item, int n_frames,
                                                        const int32_t* __restrict__ near_count,
                                                        const int4* __restrict__ near_key,
                                                        const float* __restrict__ weights,
                                                        const float* __restrict__ bias, int n_models, int features,
                                                        double clip, double eps,
                                                        const double* __restrict__ thresholds,
                                                        int32_t* __restrict__ counters, float* __restrict__ cand_score,
                                                        int4* __restrict__ cand_key, double* __restrict__ cand_s64,
                                                        const double2* __restrict__ orient, bool vec_w) {
    __shared__ RescoreShared sm;
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int total = near_count[n_frames];  // dense list of every frame's near windows
    for (int q = blockIdx.x; q < total; q += gridDim.x) {
        const int4 key = near_key[q];
        const int f = key.x / PD_MAX_LEVELS, level = key.x - f * PD_MAX_LEVELS;
        const LevelItem& it = items[first_item[f] + level];
        const int wi = key.y, wj = key.z;

        // the thread index as a value opaque to the compiler, so the gathers'
        // index arithmetic stays in the loop instead of being held in
        // registers across windows
        int tt = t;
        asm volatile("" : "+v"(tt));
        // pixels of the window + one halo pixel: every load of a thread in
        // flight together, then the LDS stores.  A window whose halo lies
        // inside the level reads aligned words (its rows start 1 byte before
        // an 8-byte boundary of a 4-byte aligned row; the last word holds the
        // halo column, so no word leaves the row); others read bytes,
        // clamped to the level.
        const bool inner = wi > 0 && wj > 0 && PD_CELL * wi + PD_WIN_H < it.h && PD_CELL * wj + PD_WIN_W < it.w;
        if (inner) {
            const auto base = it.pyr + (size_t)(PD_CELL * wi - 1) * it.pitch + (PD_CELL * wj - 4);
            uint32_t v[RS_PXW_PER_T];
#pragma unroll
            for (int k = 0; k < RS_PXW_PER_T; ++k) {
                const int e = min(tt + 256 * k, RS_PY * RS_ROW_WORDS - 1);
                const int r = e / RS_ROW_WORDS, d = e - r * RS_ROW_WORDS;
                v[k] = *reinterpret_cast<const uint32_t*>(base + (size_t)r * it.pitch + 4 * d);
            }
#pragma unroll
            for (int k = 0; k < RS_PXW_PER_T; ++k) {
                const int e = tt + 256 * k;
                if (e < RS_PY * RS_ROW_WORDS) reinterpret_cast<uint32_t*>(&sm.p.px[0][0])[e] = v[k];
            }
        } else {
            uint32_t v[RS_PX_PER_T];
#pragma unroll
            for (int k = 0; k < RS_PX_PER_T; ++k) {
                const int e = min(tt + 256 * k, RS_PY * RS_PX - 1);
                const int r = e / RS_PX, c = e - (e / RS_PX) * RS_PX;
                const int y = min(max(PD_CELL * wi - 1 + r, 0), it.h - 1);
                const int x = min(max(PD_CELL * wj - 1 + c, 0), it.w - 1);
                v[k] = it.pyr[(size_t)y * it.pitch + x];
            }
#pragma unroll
            for (int k = 0; k < RS_PX_PER_T; ++k) {
                const int e = tt + 256 * k;
                if (e < RS_PY * RS_PX) {
                    const int r = e / RS_PX, c = e - (e / RS_PX) * RS_PX;
                    sm.p.px[r][RS_PX0 + c] = (uint8_t)v[k];
                }
            }
        }
        __syncthreads();

        // LBP counts of the window's 16 x 8 cells: one run of 8 bytes per
        // plane row, read as the aligned words that hold it (each holds a
        // byte of the run, so none leaves the planes); issued here so that
        // they arrive during the votes, stored over the pixels after them
        uint32_t lw[RS_RUNS_PER_T][3];
        uint32_t loff[RS_RUNS_PER_T];
        {
            const size_t plane = (size_t)it.hc * it.wc;
#pragma unroll
            for (int k = 0; k < RS_RUNS_PER_T; ++k) {
                const int e = min(tt + 256 * k, RS_LBP_RUNS - 1);
                const int bin = e / PD_WIN_CELLS_Y, a = e - bin * PD_WIN_CELLS_Y;
                const uint8_t* p = it.lbp + bin * plane + (size_t)(wi + a) * it.wc + wj;
                loff[k] = (uint32_t)(reinterpret_cast<uintptr_t>(p) & 3);
                const uint32_t* q = reinterpret_cast<const uint32_t*>(p - loff[k]);
                lw[k][0] = q[0];
                lw[k][1] = q[1];
                lw[k][2] = loff[k] ? q[2] : 0u;
            }
        }

        // votes of cell rows 8 pass .. 8 pass + 7 into the ring of partials
        auto votes = [&](int pass) __attribute__((always_inline)) {
            const int quarter = lane >> 4;                    // pixel rows 2 quarter, 2 quarter + 1
            const int half = quarter >> 1;                    // 0: rows 0..3, 1: rows 4..7
            const int cell = wave * 16 + (lane & 15);         // of the pass's 64
            const int cy = 8 * pass + cell / PD_WIN_CELLS_X, cx = cell - (cell / PD_WIN_CELLS_X) * PD_WIN_CELLS_X;
            // acc[dy index][dx + 1][bin]; dy index 0/1 = dy -1/0 (top) or 0/+1 (bottom)
            double acc[2][3][PD_HOG_BINS];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int k = 0; k < PD_HOG_BINS; ++k) acc[a][b][k] = 0.0;
#pragma unroll 1
            for (int pr = 0; pr < 2; ++pr) {
                const int py = 2 * quarter + pr;
                const double wy0 = spatial_w(py, half - 1), wy1 = spatial_w(py, half);
                // the row's table entries, four in flight together
#pragma unroll
                for (int x4 = 0; x4 < PD_CELL; x4 += 4) {
                    double2 g[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int px = x4 + u;
                        const int r = PD_CELL * cy + py + 1, c = PD_CELL * cx + px + 1;
                        const int dx = (int)sm.p.px[r][RS_PX0 + c - 1] - (int)sm.p.px[r][RS_PX0 + c + 1];  // Algorithm 4
                        const int dy = (int)sm.p.px[r - 1][RS_PX0 + c] - (int)sm.p.px[r + 1][RS_PX0 + c];
                        const int s = dy < 0 ? -1 : 1;
                        g[u] = orient[(s * dy) * ORIENT_W + s * dx + 255];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int px = x4 + u;
                        const double tb = g[u].x, mag = g[u].y;
                        double h[PD_HOG_BINS];                         // linear vote per bin (wrap-around)
                        h[0] = fmax(0.0, 1.0 - fmin(fabs(tb), fabs(tb - 9.0)));
#pragma unroll
                        for (int k = 1; k < PD_HOG_BINS - 1; ++k) h[k] = fmax(0.0, 1.0 - fabs(tb - (double)k));
                        h[8] = fmax(0.0, 1.0 - fmin(fabs(tb - 8.0), fabs(tb + 1.0)));
                        const int q0 = px < 4 ? 0 : 1;                 // target columns q0 - 1 and q0 (as dx)
                        const double wx0 = spatial_w(px, q0 - 1), wx1 = spatial_w(px, q0);
                        const double m0 = mag * wy0, m1 = mag * wy1;
#pragma unroll
                        for (int k = 0; k < PD_HOG_BINS; ++k) {
                            acc[0][q0][k] = fma(m0 * wx0, h[k], acc[0][q0][k]);
                            acc[0][q0 + 1][k] = fma(m0 * wx1, h[k], acc[0][q0 + 1][k]);
                            acc[1][q0][k] = fma(m1 * wx0, h[k], acc[1][q0][k]);
                            acc[1][q0 + 1][k] = fma(m1 * wx1, h[k], acc[1][q0 + 1][k]);
                        }
                    }
                }
            }
            // the quarters meet: dy = -1 = top quarters' acc[0], dy = 0 = top
            // quarters' acc[1] + bottom quarters' acc[0], dy = +1 = bottom
            // quarters' acc[1]; quarter 0 stores dy = -1, quarter 1 dy = 0,
            // quarter 2 dy = +1
            double* A = sm.A[(cy % RS_RING) * PD_WIN_CELLS_X + cx];
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int k = 0; k < PD_HOG_BINS; ++k) {
                    const double p0 = acc[0][b][k] + __shfl_xor(acc[0][b][k], 16, 64);  // quarter pair sums
                    const double p1 = acc[1][b][k] + __shfl_xor(acc[1][b][k], 16, 64);
                    const double other0 = __shfl_xor(p0, 32, 64);                     // the other half's
                    if (quarter == 0) A[(0 * 3 + b) * PD_HOG_BINS + k] = p0;          // dy = -1
                    if (quarter == 1) A[(1 * 3 + b) * PD_HOG_BINS + k] = p1 + other0; // dy = 0
                    if (quarter == 2) A[(2 * 3 + b) * PD_HOG_BINS + k] = p1;          // dy = +1
                }
        };
        // blocks of block rows by0 .. (lane t < n): slot (r, c) of block (by,
        // bx) sums the partials its 4 cells aim at it; L2-Hys; stored at
        // sm.hog[t * 36 ..]
        auto blocks = [&](int by0, int n) __attribute__((always_inline)) {
            if (t >= n) return;
            const int by = by0 + t / PD_WIN_BLOCKS_X, bx = t - (t / PD_WIN_BLOCKS_X) * PD_WIN_BLOCKS_X;
            double v[PD_HOG_BLOCK];
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c)
                    for (int k = 0; k < PD_HOG_BINS; ++k) {
                        double s = 0.0;
                        for (int sy = 0; sy < 2; ++sy)
                            for (int sx = 0; sx < 2; ++sx)
                                s += sm.A[((by + sy) % RS_RING) * PD_WIN_CELLS_X + (bx + sx)]
                                         [((r - sy + 1) * 3 + (c - sx + 1)) * PD_HOG_BINS + k];
                        v[(r * 2 + c) * PD_HOG_BINS + k] = s;
                    }
            double ss = 0.0;
            for (int k = 0; k < PD_HOG_BLOCK; ++k) ss += v[k] * v[k];
            double inv = 1.0 / sqrt(ss + eps * eps);
            double ss2 = 0.0;
            for (int k = 0; k < PD_HOG_BLOCK; ++k) {
                v[k] = fmin(v[k] * inv, clip);
                ss2 += v[k] * v[k];
            }
            inv = 1.0 / sqrt(ss2 + eps * eps);
            for (int k = 0; k < PD_HOG_BLOCK; ++k) sm.hog[t * PD_HOG_BLOCK + k] = v[k] * inv;
        };
        // dot products over features [k_begin, k_end) (whole features of this
        // pass, or of the one family of an HOG-only / LBP-only detector), all
        // lanes, coalesced weights from the L2, a fixed-order reduction
        auto dot = [&](int k_begin, int k_end, int hog_base, int pass) __attribute__((always_inline)) {
            if (vec_w && n_models > 1) {
                dot_models4<8>(sm, reinterpret_cast<const float4*>(weights), n_models, k_begin / 4, k_end / 4,
                               hog_base, pass, t, wave, lane);
            } else if (n_models == 1) {
                dot_models<1>(sm, weights, 1, k_begin, k_end, hog_base, pass, t, wave, lane);
            } else {
                dot_models<8>(sm, weights, n_models, k_begin, k_end, hog_base, pass, t, wave, lane);
            }
        };
        const bool use_hog = (features & PD_FEAT_HOG) != 0, use_lbp = (features & PD_FEAT_LBP) != 0;

        // pass 1: cell rows 0..7, block rows 0..6
        votes(0);
        __syncthreads();
        blocks(0, RS_BLK1);
        __syncthreads();
        dot(0, use_hog ? RS_HOG1 : 0, 0, 0);
        // pass 2: cell rows 8..15 (over rows 0..6 of the ring, after the
        // barrier above), block rows 7..14
        votes(1);
        __syncthreads();  // the pass's partials are stored, the pixels and the pass-1 HOG values read
        blocks(PD_WIN_CELLS_Y / 2 - 1, RS_BLK2);
        {
#pragma unroll
            for (int k = 0; k < RS_RUNS_PER_T; ++k) {
                const int e = tt + 256 * k;
                if (e < RS_LBP_RUNS) {
                    const int bin = e / PD_WIN_CELLS_Y, a = e - bin * PD_WIN_CELLS_Y;
                    const uint32_t lo = __builtin_amdgcn_alignbyte(lw[k][1], lw[k][0], loff[k]);
                    const uint32_t hi = __builtin_amdgcn_alignbyte(lw[k][2], lw[k][1], loff[k]);
                    uint8_t* dst = &sm.p.lbp[(a * PD_WIN_CELLS_X) * PD_LBP_BINS + bin];
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        dst[b * PD_LBP_BINS] = (uint8_t)(lo >> (8 * b));
                        dst[(b + 4) * PD_LBP_BINS] = (uint8_t)(hi >> (8 * b));
                    }
                }
            }
        }
        __syncthreads();
        dot(use_hog ? RS_HOG1 : PD_HOG_DIM, use_lbp ? PD_FEATURE_DIM : PD_HOG_DIM, RS_HOG1, 1);
        __syncthreads();
        if (t == 0) {
            double best = 0.0;
            int bm = 0;
            for (int m = 0; m < n_models; ++m) {
                const double s1 = (sm.part[0][0][m] + sm.part[0][1][m]) + (sm.part[0][2][m] + sm.part[0][3][m]);
                const double s2 = (sm.part[1][0][m] + sm.part[1][1][m]) + (sm.part[1][2][m] + sm.part[1][3][m]);
                const double s = (s1 + s2) + (double)bias[m];
                if (m == 0 || s > best) {
                    best = s;
                    bm = m;
                }
            }
            if (best > thresholds[f]) {
                const int pos = atomicAdd(&counters[f], 1);
                if (pos < it.cand_cap) {  // always: a window is appended once at most
                    const size_t o = (size_t)it.cand_off + pos;
                    cand_score[o] = (float)best;
                    cand_key[o] = make_int4(level, wi, wj, bm);
                    cand_s64[o] = best;
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_orient_table(double2* table, hipStream_t s) {
    orient_table_kernel<<<ceil_div(ORIENT_W * ORIENT_H, 256), 256, 0, s>>>(table);
    return hipGetLastError();
}

hipError_t launch_rescore64(const LevelItem* items, const int32_t* frame_first_item, int n_frames,
                            const int32_t* near_count, const int4* near_key, const float* weights, const float* bias,
                            int n_models, int features, float clip, float eps, const double* thresholds,
                            int32_t* counters, float* cand_score, int4* cand_key, double* cand_s64,
                            const double2* orient, hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    // persistent workgroups (two per CU fit the LDS) over the dense near
    // list, whose length is read on the device
    const int grid = 1024;
    rescore64_kernel<<<grid, 256, 0, s>>>(items, frame_first_item, n_frames, near_count, near_key, weights, bias,
                                         n_models, features, (double)clip, (double)eps, thresholds, counters,
                                         cand_score, cand_key, cand_s64, orient, ((uintptr_t)weights & 15) == 0);
    return hipGetLastError();
}

}  // namespace pd
