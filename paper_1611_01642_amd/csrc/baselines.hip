// The paper's own GPU mappings of the three algorithms (Section 4), built as
// ablation baselines for the px/ns comparison of Section 5.3.  They compute
// the same results as the library's kernels (up to FP32 rounding order);
// pd_detect does not use them.
//
//  * LBP cell histograms, Naive scheme (Section 4.2): a thread per 8x8 cell
//    reads the cell's 64 codes of the LBP map (Algorithm 1, written to global
//    memory by pd_lbp_codes) and counts them in a private array.
//  * LBP cell histograms, Scalable scheme (Section 4.2, Algorithm 2): a thread
//    per pixel adds one to its cell's bin with a global atomic.
//  * HOG, Global variant (Section 4.3, Algorithms 4 and 5): a thread per pixel
//    writes magnitude and orientation to global memory; a thread per 16x16
//    block then votes every pixel of the block into the block's histogram,
//    which lives in global memory (the output itself, read-modify-write), and
//    normalises it (L2-Hys).
//  * SVM, Naive scheme (Section 4.4): a thread per window computes the dot
//    product of the window's whole feature vector with the model.
//  * SVM, warp-level scheme (Section 4.4, Algorithm 6): a wave per window;
//    lanes stride over the features, then a shuffle-tree reduction.
#include "pd_internal.h"

namespace pd {
namespace {

__constant__ LbpTable kLbpBase = make_lbp_table();

// ---- LBP ---------------------------------------------------------------------
__global__ void lbp_naive_kernel(const uint8_t* __restrict__ codes, int pitch, int wc, int hc,
                                 uint32_t* __restrict__ hist) {
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= wc * hc) return;
    const int cy = cell / wc, cx = cell - cy * wc;
    uint32_t cnt[PD_LBP_BINS];
    for (int b = 0; b < PD_LBP_BINS; ++b) cnt[b] = 0u;
    for (int py = 0; py < PD_CELL; ++py)
        for (int px = 0; px < PD_CELL; ++px)
            ++cnt[kLbpBase.bin[codes[(size_t)(PD_CELL * cy + py) * pitch + PD_CELL * cx + px]]];
    uint32_t* out = hist + (size_t)cell * PD_LBP_BINS;
    for (int b = 0; b < PD_LBP_BINS; ++b) out[b] = cnt[b];
}

__global__ void zero_u32_kernel(uint32_t* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void lbp_scatter_kernel(const uint8_t* __restrict__ codes, int pitch, int wc, int hc,
                                   uint32_t* __restrict__ hist) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= PD_CELL * wc || y >= PD_CELL * hc) return;
    const int bin = kLbpBase.bin[codes[(size_t)y * pitch + x]];
    atomicAdd(&hist[((size_t)(y / PD_CELL) * wc + x / PD_CELL) * PD_LBP_BINS + bin], 1u);
}

// ---- HOG Global ----------------------------------------------------------------
// Algorithm 4: dx = I[y][x-1] - I[y][x+1], dy = I[y-1][x] - I[y+1][x]
// (edge-clamped), magnitude and unsigned orientation in degrees.
__global__ void gradient_kernel(const uint8_t* __restrict__ img, int w, int h, int pitch, float* __restrict__ mag,
                                float* __restrict__ ang) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= w) return;
    const uint8_t* row = img + (size_t)y * pitch;
    const float dx = (float)row[max(x - 1, 0)] - (float)row[min(x + 1, w - 1)];
    const float dy = (float)img[(size_t)max(y - 1, 0) * pitch + x] - (float)img[(size_t)min(y + 1, h - 1) * pitch + x];
    float a = atan2f(dy, dx) * (180.0f / 3.14159265358979f);
    if (a < 0.0f) a += 180.0f;
    if (a >= 180.0f) a -= 180.0f;
    mag[(size_t)y * w + x] = sqrtf(dx * dx + dy * dy);
    ang[(size_t)y * w + x] = a;
}

// Algorithm 5 per block, histogram in global memory: planes [36][hb][wb],
// entry (r * 2 + c) * 9 + bin; every pixel of the 16x16 block votes into the
// two orientation bins around its angle (bin centres 10 + 20k degrees,
// wrapping) and the cell slots whose centres are within 8 pixels, with
// bilinear spatial weights; then L2-Hys on the 36 values.
__global__ void hog_global_kernel(const float* __restrict__ mag, const float* __restrict__ ang, int w, int wb,
                                  int hb, float clip, float eps, float* __restrict__ blocks) {
    const int blk = blockIdx.x * blockDim.x + threadIdx.x;
    if (blk >= wb * hb) return;
    const int by = blk / wb, bx = blk - by * wb;
    const size_t plane = (size_t)wb * hb;
    float* out = blocks + (size_t)by * wb + bx;
    for (int k = 0; k < PD_HOG_BLOCK; ++k) out[k * plane] = 0.0f;
    for (int py = 0; py < 2 * PD_CELL; ++py) {
        const float v = ((float)py + 0.5f - 4.0f) / 8.0f;  // cell-row coordinate within the block
        for (int px = 0; px < 2 * PD_CELL; ++px) {
            const float u = ((float)px + 0.5f - 4.0f) / 8.0f;
            const size_t o = (size_t)(PD_CELL * by + py) * w + PD_CELL * bx + px;
            const float m = mag[o];
            const float t = ang[o] / 20.0f - 0.5f;
            const float tf = floorf(t);
            const int b0 = ((int)tf % 9 + 9) % 9, b1 = (b0 + 1) % 9;
            const float w1 = t - tf, w0 = 1.0f - w1;
            for (int r = 0; r < 2; ++r) {
                const float wy = fmaxf(0.0f, 1.0f - fabsf(v - (float)r));
                if (wy == 0.0f) continue;
                for (int c = 0; c < 2; ++c) {
                    const float wx = fmaxf(0.0f, 1.0f - fabsf(u - (float)c));
                    if (wx == 0.0f) continue;
                    const float mw = m * wy * wx;
                    out[((r * 2 + c) * PD_HOG_BINS + b0) * plane] += mw * w0;
                    out[((r * 2 + c) * PD_HOG_BINS + b1) * plane] += mw * w1;
                }
            }
        }
    }
    float ss = 0.0f;
    for (int k = 0; k < PD_HOG_BLOCK; ++k) ss += out[k * plane] * out[k * plane];
    const float inv = 1.0f / sqrtf(ss + eps * eps);
    float ss2 = 0.0f;
    for (int k = 0; k < PD_HOG_BLOCK; ++k) {
        const float x = fminf(out[k * plane] * inv, clip);
        out[k * plane] = x;
        ss2 += x * x;
    }
    const float inv2 = 1.0f / sqrtf(ss2 + eps * eps);
    for (int k = 0; k < PD_HOG_BLOCK; ++k) out[k * plane] *= inv2;
}

// ---- SVM -----------------------------------------------------------------------
// Feature k of window (i, j): HOG value (a, b, c) for k < 3780, else the LBP
// count (a, b, c) (the window-vector order of pd_score_windows).
__device__ __forceinline__ float window_feature(const float* __restrict__ blocks, const uint8_t* __restrict__ cells,
                                                int wc, int hc, int i, int j, int k) {
    if (k < PD_HOG_DIM) {
        const int c = k % PD_HOG_BLOCK, ab = k / PD_HOG_BLOCK;
        const int a = ab / PD_WIN_BLOCKS_X, b = ab - a * PD_WIN_BLOCKS_X;
        return blocks[((size_t)c * (hc - 1) + i + a) * (wc - 1) + j + b];
    }
    const int q = k - PD_HOG_DIM;
    const int c = q % PD_LBP_BINS, ab = q / PD_LBP_BINS;
    const int a = ab / PD_WIN_CELLS_X, b = ab - a * PD_WIN_CELLS_X;
    return (float)cells[((size_t)c * hc + i + a) * wc + j + b];
}

__global__ void svm_naive_kernel(const float* __restrict__ blocks, const uint8_t* __restrict__ cells, int wc, int hc,
                                 const float* __restrict__ weights, const float* __restrict__ bias, int n_models,
                                 float* __restrict__ scores) {
    const int nx = wc - PD_WIN_CELLS_X + 1, ny = hc - PD_WIN_CELLS_Y + 1;
    const int win = blockIdx.x * blockDim.x + threadIdx.x;
    if (win >= nx * ny) return;
    const int i = win / nx, j = win - i * nx;
    for (int m = 0; m < n_models; ++m) {
        const float* wm = weights + (size_t)m * PD_FEATURE_DIM;
        float s = 0.0f;
        for (int k = 0; k < PD_FEATURE_DIM; ++k) s = fmaf(window_feature(blocks, cells, wc, hc, i, j, k), wm[k], s);
        scores[(size_t)m * nx * ny + win] = s + bias[m];
    }
}

__global__ void __launch_bounds__(256) svm_wave_kernel(const float* __restrict__ blocks,
                                                       const uint8_t* __restrict__ cells, int wc, int hc,
                                                       const float* __restrict__ weights,
                                                       const float* __restrict__ bias, int n_models,
                                                       float* __restrict__ scores) {
    const int nx = wc - PD_WIN_CELLS_X + 1, ny = hc - PD_WIN_CELLS_Y + 1;
    const int win = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (win >= nx * ny) return;  // the whole wave leaves together
    const int i = win / nx, j = win - i * nx;
    for (int m = 0; m < n_models; ++m) {
        const float* wm = weights + (size_t)m * PD_FEATURE_DIM;
        float s = 0.0f;
        for (int k = lane; k < PD_FEATURE_DIM; k += 64) s = fmaf(window_feature(blocks, cells, wc, hc, i, j, k), wm[k], s);
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) scores[(size_t)m * nx * ny + win] = s + bias[m];
    }
}

}  // namespace

hipError_t launch_lbp_naive(const uint8_t* codes, int pitch, int wc, int hc, uint32_t* hist, hipStream_t s) {
    const int n = wc * hc;
    if (n <= 0) return hipSuccess;
    lbp_naive_kernel<<<ceil_div(n, 256), 256, 0, s>>>(codes, pitch, wc, hc, hist);
    return hipGetLastError();
}

hipError_t launch_lbp_scatter(const uint8_t* codes, int pitch, int wc, int hc, uint32_t* hist, hipStream_t s) {
    const int64_t n = (int64_t)wc * hc * PD_LBP_BINS;
    if (n <= 0) return hipSuccess;
    zero_u32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(hist, n);
    lbp_scatter_kernel<<<dim3(ceil_div(PD_CELL * wc, 256), PD_CELL * hc), 256, 0, s>>>(codes, pitch, wc, hc, hist);
    return hipGetLastError();
}

hipError_t launch_hog_global(const uint8_t* img, int w, int h, int pitch, float clip, float eps, float* grad,
                             float* blocks, hipStream_t s) {
    const int wb = w / PD_CELL - 1, hb = h / PD_CELL - 1;
    float* mag = grad;
    float* ang = grad + (size_t)w * h;
    gradient_kernel<<<dim3(ceil_div(w, 256), h), 256, 0, s>>>(img, w, h, pitch, mag, ang);
    if (wb > 0 && hb > 0)
        hog_global_kernel<<<ceil_div(wb * hb, 64), 64, 0, s>>>(mag, ang, w, wb, hb, clip, eps, blocks);
    return hipGetLastError();
}

hipError_t launch_svm_naive(const float* blocks, const uint8_t* cells, int wc, int hc, const float* w,
                            const float* bias, int n_models, float* scores, hipStream_t s) {
    const int n = (wc - PD_WIN_CELLS_X + 1) * (hc - PD_WIN_CELLS_Y + 1);
    svm_naive_kernel<<<ceil_div(n, 64), 64, 0, s>>>(blocks, cells, wc, hc, w, bias, n_models, scores);
    return hipGetLastError();
}

hipError_t launch_svm_wave(const float* blocks, const uint8_t* cells, int wc, int hc, const float* w,
                           const float* bias, int n_models, float* scores, hipStream_t s) {
    const int n = (wc - PD_WIN_CELLS_X + 1) * (hc - PD_WIN_CELLS_Y + 1);
    svm_wave_kernel<<<ceil_div(n, 4), 256, 0, s>>>(blocks, cells, wc, hc, w, bias, n_models, scores);
    return hipGetLastError();
}

}  // namespace pd
