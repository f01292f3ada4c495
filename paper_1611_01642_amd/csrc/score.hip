// Sliding-window linear-SVM scoring (Section 4.4, Algorithm 6) in FP32 on the
// vector ALUs, one image per call (pd_score_windows and the single-image
// forms; batched detection scores on the matrix cores, score32.hip).
//
// The score of window (i, j) is a 2-D correlation of the feature planes with
// the model:  s(i,j) = sum_c sum_a sum_b F_c[i+a][j+b] * W[a][b][c] + bias.
// Algorithm 6 gives each window a warp that re-reads the window's whole
// feature vector.  Here one wave64 owns a tile of 64 adjacent window columns
// (one per lane) x R window rows (registers; R = 8 or 16).  For each feature plane c the
// wave stages the tile's (R + 14 or 15) x (64 + 6 or 7) patch in its own
// LDS region (coalesced loads of the next plane are in flight while the
// current one is used), then every patch value a lane reads from LDS serves up
// to R windows of its column.  Weights are wave-uniform (scalar loads).
// FP32 products and FP32 sums in a fixed order.
#include "pd_internal.h"

namespace pd {
namespace {

// Patch geometry for R window rows per lane group of L lanes (64 / L groups
// per wave, each on its own row chunk, all on the same L window columns).
template <int R, int L = SC_W>
struct Patch {
    static constexpr int G = SC_W / L;
    static constexpr int HOG_PR = R + PD_WIN_BLOCKS_Y - 1;  // patch rows per group
    static constexpr int HOG_PC = L + PD_WIN_BLOCKS_X - 1;  // patch columns
    static constexpr int LBP_PR = R + PD_WIN_CELLS_Y - 1;
    static constexpr int LBP_PC = L + PD_WIN_CELLS_X - 1;
    static constexpr int HOG_N = G * HOG_PR * HOG_PC, LBP_N = G * LBP_PR * LBP_PC;
    static constexpr int HOG_PQ = (HOG_N + 63) / 64;  // patch values per lane
    static constexpr int LBP_PQ = (LBP_N + 63) / 64;
    static constexpr int SIZE = HOG_N > LBP_N ? HOG_N : LBP_N;
};

// R window rows per lane from row (ty + group) * STEP: a tile laid out on a
// grid of STEP rows whose valid rows fit in R < STEP computes only those.
template <int FEAT, int R, int L = SC_W, int STEP = R>
__device__ __forceinline__ void score_tile(gptr<const float> __restrict__ hog, gptr<const uint8_t> __restrict__ lbp,
                                           int wc, int hc, const float* __restrict__ wt, float bias,
                                           gptr<float> __restrict__ out,
                                           int ty, int tx, int lane, float* __restrict__ patch) {
    using PG = Patch<R, L>;
    constexpr int HOG_PR = PG::HOG_PR, HOG_PC = PG::HOG_PC, HOG_PQ = PG::HOG_PQ, HOG_N = PG::HOG_N;
    constexpr int LBP_PR = PG::LBP_PR, LBP_PC = PG::LBP_PC, LBP_PQ = PG::LBP_PQ, LBP_N = PG::LBP_N;
    const int hb = hc - 1, wb = wc - 1;
    const int ny = hc - PD_WIN_CELLS_Y + 1, nx = wc - PD_WIN_CELLS_X + 1;
    const int g = lane / L, li = lane % L;  // group and column within it
    const int j0 = tx * SC_W;
    float acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0f;

    if (FEAT & PD_FEAT_HOG) {
        const size_t plane = (size_t)hb * wb;
        // clamped byte offsets in a plane of this lane's patch values; the
        // loads are raw buffer loads with the plane's byte offset as a scalar,
        // so no address arithmetic is done per value
        const auto rsrc = planes_rsrc(hog, (uint64_t)PD_HOG_BLOCK * plane * 4);
        uint32_t off[HOG_PQ];
#pragma unroll
        for (int q = 0; q < HOG_PQ; ++q) {
            const int e = min(lane + 64 * q, HOG_N - 1);
            const int gq = e / (HOG_PR * HOG_PC), rem = e - gq * (HOG_PR * HOG_PC);
            const int row = rem / HOG_PC, col = rem - (rem / HOG_PC) * HOG_PC;
            off[q] = 4u * (uint32_t)(min((ty + gq) * STEP + row, hb - 1) * wb + min(j0 + col, wb - 1));
        }
        float pre[HOG_PQ];
#pragma unroll
        for (int q = 0; q < HOG_PQ; ++q)
            pre[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, off[q], 0, 0));
        for (int c = 0; c < PD_HOG_BLOCK; ++c) {
#pragma unroll
            for (int q = 0; q < HOG_PQ; ++q)
                if (lane + 64 * q < HOG_N) patch[lane + 64 * q] = pre[q];
            if (c + 1 < PD_HOG_BLOCK) {
                const uint32_t pofs = (uint32_t)((c + 1) * plane * 4);
#pragma unroll
                for (int q = 0; q < HOG_PQ; ++q)
                    pre[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, off[q], pofs, 0));
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll 1
            for (int b = 0; b < PD_WIN_BLOCKS_X; ++b) {
                float wa[PD_WIN_BLOCKS_Y];
#pragma unroll
                for (int a = 0; a < PD_WIN_BLOCKS_Y; ++a) wa[a] = wt[(a * PD_WIN_BLOCKS_X + b) * PD_HOG_BLOCK + c];
                const float* pr = patch + g * (HOG_PR * HOG_PC) + li + b;
#pragma unroll
                for (int y = 0; y < HOG_PR; ++y) {
                    const float v = pr[y * HOG_PC];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int a = y - r;
                        if (a >= 0 && a < PD_WIN_BLOCKS_Y) acc[r] = fmaf(v, wa[a], acc[r]);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (FEAT & PD_FEAT_LBP) {
        const size_t plane = (size_t)hc * wc;
        const float* wl = wt + PD_HOG_DIM;
        const auto rsrc = planes_rsrc(lbp, (uint64_t)PD_LBP_BINS * plane);
        uint32_t off[LBP_PQ];  // clamped byte offsets in a plane (as for HOG)
#pragma unroll
        for (int q = 0; q < LBP_PQ; ++q) {
            const int e = min(lane + 64 * q, LBP_N - 1);
            const int gq = e / (LBP_PR * LBP_PC), rem = e - gq * (LBP_PR * LBP_PC);
            const int row = rem / LBP_PC, col = rem - (rem / LBP_PC) * LBP_PC;
            off[q] = (uint32_t)(min((ty + gq) * STEP + row, hc - 1) * wc + min(j0 + col, wc - 1));
        }
        uint32_t pre[LBP_PQ];
#pragma unroll
        for (int q = 0; q < LBP_PQ; ++q) pre[q] = __builtin_amdgcn_raw_buffer_load_b8(rsrc, off[q], 0, 0);
        for (int c = 0; c < PD_LBP_BINS; ++c) {
#pragma unroll
            for (int q = 0; q < LBP_PQ; ++q)
                if (lane + 64 * q < LBP_N) patch[lane + 64 * q] = (float)pre[q];
            if (c + 1 < PD_LBP_BINS) {
                const uint32_t pofs = (uint32_t)((c + 1) * plane);
#pragma unroll
                for (int q = 0; q < LBP_PQ; ++q) pre[q] = __builtin_amdgcn_raw_buffer_load_b8(rsrc, off[q], pofs, 0);
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll 1
            for (int b = 0; b < PD_WIN_CELLS_X; ++b) {
                float wa[PD_WIN_CELLS_Y];
#pragma unroll
                for (int a = 0; a < PD_WIN_CELLS_Y; ++a) wa[a] = wl[(a * PD_WIN_CELLS_X + b) * PD_LBP_BINS + c];
                const float* pr = patch + g * (LBP_PR * LBP_PC) + li + b;
#pragma unroll
                for (int y = 0; y < LBP_PR; ++y) {
                    const float v = pr[y * LBP_PC];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int a = y - r;
                        if (a >= 0 && a < PD_WIN_CELLS_Y) acc[r] = fmaf(v, wa[a], acc[r]);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    const int i0 = (ty + g) * STEP;
    const int j = j0 + li;
    if (j < nx) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = i0 + r;
            if (i < ny) out[(size_t)i * nx + j] = acc[r] + bias;
        }
    }
}

template <int FEAT>
__global__ void __launch_bounds__(256) score_single_kernel(LevelItem it, const float* __restrict__ wt,
                                                           const float* __restrict__ bias, int n_models) {
    __shared__ float patches[SC_WAVES][Patch<SC_R>::SIZE];
    const int wave = blockIdx.x * SC_WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntx = score_tiles_x(it.nx), nty = score_tiles_y(it.ny);
    const int per_model = ntx * nty;
    if (wave >= per_model * n_models) return;
    const int m = wave / per_model;
    const int local = wave - m * per_model;
    score_tile<FEAT, SC_R>(gmem(it.hog), gmem(it.lbp), it.wc, it.hc, wt + (size_t)m * PD_FEATURE_DIM, bias[m],
                           gmem(it.scores) + (size_t)m * it.ny * it.nx, local / ntx, local % ntx, threadIdx.x & 63,
                           patches[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)]);
}

template <int FEAT>
hipError_t score_single(const LevelItem& it, const float* w, const float* b, int m, hipStream_t s) {
    const int waves = score_tiles_x(it.nx) * score_tiles_y(it.ny) * m;
    score_single_kernel<FEAT><<<ceil_div(waves, SC_WAVES), 256, 0, s>>>(it, w, b, m);
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

}  // namespace pd
