// Sliding-window linear-SVM scoring (Section 4.4, Algorithm 6) in FP32.
//
// The score of window (i, j) is a 2-D correlation of the feature planes with
// the model:  s(i,j) = sum_c sum_a sum_b F_c[i+a][j+b] * W[a][b][c] + bias.
// Algorithm 6 gives each window a warp that re-reads the window's whole
// feature vector; here one wave64 owns 64 adjacent window columns (one per
// lane) and SC_R window rows (registers), so every feature value a lane loads
// serves up to 15 (HOG) or 16 (LBP) windows of its column, and the loads of a
// wave are 64 consecutive floats/bytes of one plane row (coalesced).  Weights
// are wave-uniform (scalar loads).  FP32 products, FP32 sums in a fixed order.
#include "pd_internal.h"

namespace pd {
namespace {

template <int FEAT>
__device__ void score_tile(const float* __restrict__ hog, const uint8_t* __restrict__ lbp, int wc, int hc,
                           const float* __restrict__ wt, float bias, float* __restrict__ out, int ty,
                           int tx, int lane) {
    const int hb = hc - 1, wb = wc - 1;
    const int ny = hc - PD_WIN_CELLS_Y + 1, nx = wc - PD_WIN_CELLS_X + 1;
    const int i0 = ty * SC_R;
    const int j = tx * SC_W + lane;
    const int jj = min(j, nx - 1);   // lanes past the last column load valid data
    float acc[SC_R];
#pragma unroll
    for (int r = 0; r < SC_R; ++r) acc[r] = 0.0f;

    if (FEAT & PD_FEAT_HOG) {
        const size_t plane = (size_t)hb * wb;
        for (int c = 0; c < PD_HOG_BLOCK; ++c) {
            const float* fp = hog + c * plane + jj;
            for (int b = 0; b < PD_WIN_BLOCKS_X; ++b) {
                float wa[PD_WIN_BLOCKS_Y];
#pragma unroll
                for (int a = 0; a < PD_WIN_BLOCKS_Y; ++a)
                    wa[a] = wt[(a * PD_WIN_BLOCKS_X + b) * PD_HOG_BLOCK + c];
#pragma unroll
                for (int y = 0; y < SC_R + PD_WIN_BLOCKS_Y - 1; ++y) {
                    const int row = min(i0 + y, hb - 1);
                    const float v = fp[(size_t)row * wb + b];
#pragma unroll
                    for (int r = 0; r < SC_R; ++r) {
                        const int a = y - r;
                        if (a >= 0 && a < PD_WIN_BLOCKS_Y) acc[r] = fmaf(v, wa[a], acc[r]);
                    }
                }
            }
        }
    }
    if (FEAT & PD_FEAT_LBP) {
        const size_t plane = (size_t)hc * wc;
        const float* wl = wt + PD_HOG_DIM;
        for (int c = 0; c < PD_LBP_BINS; ++c) {
            const uint8_t* fp = lbp + c * plane + jj;
            for (int b = 0; b < PD_WIN_CELLS_X; ++b) {
                float wa[PD_WIN_CELLS_Y];
#pragma unroll
                for (int a = 0; a < PD_WIN_CELLS_Y; ++a)
                    wa[a] = wl[(a * PD_WIN_CELLS_X + b) * PD_LBP_BINS + c];
#pragma unroll
                for (int y = 0; y < SC_R + PD_WIN_CELLS_Y - 1; ++y) {
                    const int row = min(i0 + y, hc - 1);
                    const float v = (float)fp[(size_t)row * wc + b];
#pragma unroll
                    for (int r = 0; r < SC_R; ++r) {
                        const int a = y - r;
                        if (a >= 0 && a < PD_WIN_CELLS_Y) acc[r] = fmaf(v, wa[a], acc[r]);
                    }
                }
            }
        }
    }
    if (j < nx) {
#pragma unroll
        for (int r = 0; r < SC_R; ++r) {
            const int i = i0 + r;
            if (i < ny) out[(size_t)i * nx + j] = acc[r] + bias;
        }
    }
}

template <int FEAT>
__global__ void __launch_bounds__(256) score_single_kernel(LevelItem it, const float* __restrict__ wt,
                                                           const float* __restrict__ bias, int n_models) {
    const int wave = blockIdx.x * SC_WAVES + (threadIdx.x >> 6);
    const int ntx = score_tiles_x(it.nx), nty = score_tiles_y(it.ny);
    const int per_model = ntx * nty;
    if (wave >= per_model * n_models) return;
    const int m = wave / per_model;
    const int local = wave - m * per_model;
    score_tile<FEAT>(it.hog, it.lbp, it.wc, it.hc, wt + (size_t)m * PD_FEATURE_DIM, bias[m],
                     it.scores + (size_t)m * it.ny * it.nx, local / ntx, local % ntx, threadIdx.x & 63);
}

// Tile.pad carries the model index.
template <int FEAT>
__global__ void __launch_bounds__(256) score_table_kernel(const LevelItem* __restrict__ items,
                                                          const Tile* __restrict__ tiles, int n_tiles,
                                                          const float* __restrict__ wt,
                                                          const float* __restrict__ bias) {
    const int wave = blockIdx.x * SC_WAVES + (threadIdx.x >> 6);
    if (wave >= n_tiles) return;
    const Tile tl = tiles[wave];
    const LevelItem& it = items[tl.item];
    const int m = tl.pad;
    score_tile<FEAT>(it.hog, it.lbp, it.wc, it.hc, wt + (size_t)m * PD_FEATURE_DIM, bias[m],
                     it.scores + (size_t)m * it.ny * it.nx, tl.ty, tl.tx, threadIdx.x & 63);
}

template <int FEAT>
hipError_t score_single(const LevelItem& it, const float* w, const float* b, int m, hipStream_t s) {
    const int waves = score_tiles_x(it.nx) * score_tiles_y(it.ny) * m;
    score_single_kernel<FEAT><<<ceil_div(waves, SC_WAVES), 256, 0, s>>>(it, w, b, m);
    return hipGetLastError();
}

template <int FEAT>
hipError_t score_table(const LevelItem* items, const Tile* tiles, int n, const float* w, const float* b,
                       hipStream_t s) {
    score_table_kernel<FEAT><<<ceil_div(n, SC_WAVES), 256, 0, s>>>(items, tiles, n, w, b);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_score_single(const LevelItem& it, const float* w, const float* bias, int n_models,
                               int features, hipStream_t s) {
    if (it.nx <= 0 || it.ny <= 0 || n_models <= 0) return hipSuccess;
    switch (features & (PD_FEAT_HOG | PD_FEAT_LBP)) {
        case PD_FEAT_HOG: return score_single<PD_FEAT_HOG>(it, w, bias, n_models, s);
        case PD_FEAT_LBP: return score_single<PD_FEAT_LBP>(it, w, bias, n_models, s);
        default: return score_single<PD_FEAT_HOG | PD_FEAT_LBP>(it, w, bias, n_models, s);
    }
}

hipError_t launch_score_table(const LevelItem* items, const Tile* tiles, int n_tiles, const float* w,
                              const float* bias, int n_models, int features, hipStream_t s) {
    (void)n_models;
    if (n_tiles <= 0) return hipSuccess;
    switch (features & (PD_FEAT_HOG | PD_FEAT_LBP)) {
        case PD_FEAT_HOG: return score_table<PD_FEAT_HOG>(items, tiles, n_tiles, w, bias, s);
        case PD_FEAT_LBP: return score_table<PD_FEAT_LBP>(items, tiles, n_tiles, w, bias, s);
        default: return score_table<PD_FEAT_HOG | PD_FEAT_LBP>(items, tiles, n_tiles, w, bias, s);
    }
}

}  // namespace pd
