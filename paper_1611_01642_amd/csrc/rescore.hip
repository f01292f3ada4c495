// FP64 rescoring of near-threshold windows.
//
// After BF16 scoring, a window whose score lies within `margin` of its
// frame's threshold cannot be classified safely (Section 4.4: positive iff
// the distance to the hyper-plane exceeds the threshold).  This kernel
// recomputes such a window's features from the pixels of its pyramid level in
// FP64 -- gradients (Algorithm 4) with the device's double atan2, trilinear
// HOG votes (Algorithm 5) as per-cell direction partials, L2-Hys -- takes its
// LBP counts (exact integers) from the feature planes, and scores every model
// in FP64 with the FP32 weights.  A window whose FP64 score (max over models)
// exceeds the threshold is appended to the frame's candidate list.
//
// One workgroup per near window: lanes 0..127 own the window's 16x8 cells
// (pixel work and per-cell partials in LDS, no atomics); then lanes 0..104
// assemble the 15x7 blocks and lanes 128..255 take the 16x8 LBP cells; the
// per-lane partial dot products are reduced in a fixed order.
#include "pd_internal.h"

namespace pd {
namespace {

constexpr int RS_PY = PD_WIN_H + 2;  // 130 pixel rows incl. halo
constexpr int RS_PX = PD_WIN_W + 2;  // 66 pixel columns incl. halo
constexpr int RS_CELLS = PD_WIN_CELLS_Y * PD_WIN_CELLS_X;  // 128

struct RescoreShared {
    uint8_t px[RS_PY][RS_PX + 2];
    double A[RS_CELLS][81];            // per cell: 3x3 target cells x 9 bins
    double part[256][8];               // per lane, per model
    int take;
};

__device__ double spatial_w(int p, int d) {  // pixel offset p in its cell towards cell d in {-1,0,1}
    const double w = 1.0 - fabs((double)p + 0.5 - (8.0 * d + 4.0)) / 8.0;
    return w > 0.0 ? w : 0.0;
}

__global__ void __launch_bounds__(256) rescore64_kernel(const LevelItem* __restrict__ items,
                                                        const int32_t* __restrict__ first_item, int n_frames,
                                                        const int32_t* __restrict__ near_count,
                                                        const int4* __restrict__ near_key,
                                                        const float* __restrict__ weights,
                                                        const float* __restrict__ bias, int n_models, double clip,
                                                        double eps, const double* __restrict__ thresholds,
                                                        int32_t* __restrict__ counters, float* __restrict__ cand_score,
                                                        int4* __restrict__ cand_key, double* __restrict__ cand_s64) {
    __shared__ RescoreShared sm;
    const int t = threadIdx.x;
    const int total = near_count[n_frames];  // dense list of every frame's near windows
    for (int q = blockIdx.x; q < total; q += gridDim.x) {
        const int4 key = near_key[q];
        const int f = key.x / PD_MAX_LEVELS, level = key.x - f * PD_MAX_LEVELS;
        const LevelItem& it = items[first_item[f] + level];
        const int wi = key.y, wj = key.z;

        // pixels of the window + one halo pixel, clamped to the level
        for (int e = t; e < RS_PY * RS_PX; e += 256) {
            const int r = e / RS_PX, c = e - (e / RS_PX) * RS_PX;
            const int y = min(max(PD_CELL * wi - 1 + r, 0), it.h - 1);
            const int x = min(max(PD_CELL * wj - 1 + c, 0), it.w - 1);
            sm.px[r][c] = it.pyr[(size_t)y * it.pitch + x];
        }
        __syncthreads();

        if (t < RS_CELLS) {
            double* A = sm.A[t];
            for (int k = 0; k < 81; ++k) A[k] = 0.0;
            const int cy = t / PD_WIN_CELLS_X, cx = t - (t / PD_WIN_CELLS_X) * PD_WIN_CELLS_X;
            for (int py = 0; py < PD_CELL; ++py) {
                for (int px = 0; px < PD_CELL; ++px) {
                    const int r = PD_CELL * cy + py + 1, c = PD_CELL * cx + px + 1;
                    const int dx = (int)sm.px[r][c - 1] - (int)sm.px[r][c + 1];   // Algorithm 4
                    const int dy = (int)sm.px[r - 1][c] - (int)sm.px[r + 1][c];
                    const double mag = sqrt((double)(dx * dx + dy * dy));
                    double ang = atan2((double)dy, (double)dx) * 57.295779513082320876798154814105;
                    if (ang < 0.0) ang += 180.0;
                    if (ang >= 180.0) ang -= 180.0;
                    const double tb = ang / 20.0 - 0.5;
                    const double fl = floor(tb);
                    int b0 = (int)fl % PD_HOG_BINS;
                    if (b0 < 0) b0 += PD_HOG_BINS;
                    const int b1 = (b0 + 1) % PD_HOG_BINS;
                    const double w1 = tb - fl, w0 = 1.0 - w1;
                    for (int ddy = -1; ddy <= 1; ++ddy) {
                        const double wy = spatial_w(py, ddy);
                        if (wy == 0.0) continue;
                        for (int ddx = -1; ddx <= 1; ++ddx) {
                            const double wx = spatial_w(px, ddx);
                            if (wx == 0.0) continue;
                            const int dir = (ddy + 1) * 3 + (ddx + 1);
                            A[dir * PD_HOG_BINS + b0] += mag * wy * wx * w0;
                            A[dir * PD_HOG_BINS + b1] += mag * wy * wx * w1;
                        }
                    }
                }
            }
        }
        __syncthreads();

        double part[8];
        for (int m = 0; m < 8; ++m) part[m] = 0.0;
        if (t < PD_WIN_BLOCKS_Y * PD_WIN_BLOCKS_X) {
            const int by = t / PD_WIN_BLOCKS_X, bx = t - (t / PD_WIN_BLOCKS_X) * PD_WIN_BLOCKS_X;
            double v[PD_HOG_BLOCK];
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c)
                    for (int k = 0; k < PD_HOG_BINS; ++k) {
                        double s = 0.0;
                        for (int sy = 0; sy < 2; ++sy)
                            for (int sx = 0; sx < 2; ++sx)
                                s += sm.A[(by + sy) * PD_WIN_CELLS_X + (bx + sx)][((r - sy + 1) * 3 + (c - sx + 1)) *
                                                                                   PD_HOG_BINS + k];
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
            for (int m = 0; m < n_models; ++m) {
                const float* w = weights + (size_t)m * PD_FEATURE_DIM + (by * PD_WIN_BLOCKS_X + bx) * PD_HOG_BLOCK;
                double s = 0.0;
                for (int k = 0; k < PD_HOG_BLOCK; ++k) s += (v[k] * inv) * (double)w[k];
                part[m] = s;
            }
        } else if (t >= 128) {
            const int u = t - 128;
            const int a = u / PD_WIN_CELLS_X, b = u - (u / PD_WIN_CELLS_X) * PD_WIN_CELLS_X;
            const size_t plane = (size_t)it.hc * it.wc;
            const uint8_t* cnt = it.lbp + (size_t)(wi + a) * it.wc + (wj + b);
            for (int m = 0; m < n_models; ++m) {
                const float* w = weights + (size_t)m * PD_FEATURE_DIM + PD_HOG_DIM + (a * PD_WIN_CELLS_X + b) * PD_LBP_BINS;
                double s = 0.0;
                for (int c = 0; c < PD_LBP_BINS; ++c) s += (double)cnt[c * plane] * (double)w[c];
                part[m] = s;
            }
        }
        for (int m = 0; m < 8; ++m) sm.part[t][m] = part[m];
        __syncthreads();
        for (int stride = 128; stride > 0; stride >>= 1) {
            if (t < stride)
                for (int m = 0; m < 8; ++m) sm.part[t][m] += sm.part[t + stride][m];
            __syncthreads();
        }
        if (t == 0) {
            double best = sm.part[0][0] + (double)bias[0];
            int bm = 0;
            for (int m = 1; m < n_models; ++m) {
                const double s = sm.part[0][m] + (double)bias[m];
                if (s > best) {
                    best = s;
                    bm = m;
                }
            }
            if (best > thresholds[f]) {
                const int pos = atomicAdd(&counters[f], 1);
                if (pos < PD_MAX_CANDIDATES) {
                    const size_t o = (size_t)f * PD_MAX_CANDIDATES + pos;
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

hipError_t launch_rescore64(const LevelItem* items, const int32_t* frame_first_item, int n_frames,
                            const int32_t* near_count, const int4* near_key, const float* weights, const float* bias,
                            int n_models, float clip, float eps, const double* thresholds, int32_t* counters,
                            float* cand_score, int4* cand_key, double* cand_s64, hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    const int grid = min(n_frames * MAX_NEAR, 1024);
    rescore64_kernel<<<grid, 256, 0, s>>>(items, frame_first_item, n_frames, near_count, near_key, weights, bias,
                                         n_models, (double)clip, (double)eps, thresholds, counters, cand_score,
                                         cand_key, cand_s64);
    return hipGetLastError();
}

}  // namespace pd
