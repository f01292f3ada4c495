// LBP block histograms (Section 4.2, Algorithm 3) and the cell-level form of
// a model over LBP block histograms.
//
// A block histogram is the plain sum of the four 8x8 cell histograms of a
// 16x16 block (blocks overlap by one cell).  lbp_blocks_kernel computes it
// from the cell planes: one wave per output row (image, bin, block row),
// lanes along the row; the two cell rows it reads are coalesced byte runs,
// the uint16 output row a coalesced store (a block counts up to 256).
//
// Because the reduction is a plain sum, a linear model over block histograms
// scores every window exactly as the cell-level model whose LBP weight for a
// window cell is the sum of the weights of the window blocks containing it.
// fold_lbp_weights_kernel builds that model, one thread per output weight,
// summing its (up to four) block weights in a fixed order; the detector then
// runs on cell histograms unchanged and the blocks are never materialised.
#include "pd_internal.h"

namespace pd {
namespace {

constexpr int LB_WAVES = 4;  // output rows per workgroup

__global__ void __launch_bounds__(256) lbp_blocks_kernel(const uint8_t* __restrict__ cells, int n_rows, int hc,
                                                         int wc, uint16_t* __restrict__ blocks) {
    const int row = blockIdx.x * LB_WAVES + (threadIdx.x >> 6);  // ((image * 59) + bin) * hb + y
    if (row >= n_rows) return;
    const int hb = hc - 1, wb = wc - 1;
    const int plane = row / hb, y = row - plane * hb;
    const uint8_t* top = cells + ((size_t)plane * hc + y) * wc;
    const uint8_t* bot = top + wc;
    uint16_t* out = blocks + (size_t)row * wb;
    for (int x = threadIdx.x & 63; x < wb; x += 64)
        out[x] = (uint16_t)(top[x] + top[x + 1] + bot[x] + bot[x + 1]);
}

__global__ void __launch_bounds__(256) fold_lbp_weights_kernel(const float* __restrict__ wb, int n_models,
                                                               float* __restrict__ w) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_models * PD_FEATURE_DIM) return;
    const int m = e / PD_FEATURE_DIM, q = e - m * PD_FEATURE_DIM;
    const float* src = wb + (size_t)m * PD_BLOCK_MODEL_DIM;
    if (q < PD_HOG_DIM) {
        w[e] = src[q];
        return;
    }
    const int r = q - PD_HOG_DIM;
    const int k = r % PD_LBP_BINS, cell = r / PD_LBP_BINS;
    const int a = cell / PD_WIN_CELLS_X, b = cell - a * PD_WIN_CELLS_X;
    float s = 0.0f;
#pragma unroll
    for (int da = 1; da >= 0; --da)
#pragma unroll
        for (int db = 1; db >= 0; --db) {
            const int a2 = a - da, b2 = b - db;  // window block (a2, b2) holds cell (a, b)
            if (a2 >= 0 && a2 < PD_WIN_BLOCKS_Y && b2 >= 0 && b2 < PD_WIN_BLOCKS_X)
                s += src[PD_HOG_DIM + (a2 * PD_WIN_BLOCKS_X + b2) * PD_LBP_BINS + k];
        }
    w[e] = s;
}

}  // namespace

hipError_t launch_lbp_blocks(const uint8_t* cells, int n, int hc, int wc, uint16_t* blocks, hipStream_t s) {
    const int n_rows = n * PD_LBP_BINS * (hc - 1);
    lbp_blocks_kernel<<<ceil_div(n_rows, LB_WAVES), 256, 0, s>>>(cells, n_rows, hc, wc, blocks);
    return hipGetLastError();
}

hipError_t launch_fold_lbp_weights(const float* wb, int n_models, float* w, hipStream_t s) {
    fold_lbp_weights_kernel<<<ceil_div(n_models * PD_FEATURE_DIM, 256), 256, 0, s>>>(wb, n_models, w);
    return hipGetLastError();
}

}  // namespace pd
