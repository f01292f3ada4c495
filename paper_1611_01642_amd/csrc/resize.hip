// Pyramid resize (Section 4.1 step 2, Section 4.4): every level is resampled
// from the level-0 image with pixel-centre-aligned bilinear interpolation in
// Q8 fixed point, rounded half up.  All arithmetic is integer, so results are
// exact.  One workgroup writes a 256 x 16 pixel tile of one level; the Q8
// coordinates of the tile's columns and rows are computed once per tile in
// LDS (they need a 64-bit division).
#include "pd_internal.h"

namespace pd {
namespace {

// Q8 source coordinate of output sample `x` along an axis of n0 -> nk
// samples: ((2x + 1) n0 - nk) * 128 / nk, split into index and fraction.
__device__ inline uint32_t q8_coord(int x, int n0, int nk) {
    int64_t num = (int64_t)(2 * x + 1) * n0 - nk;
    int64_t s = (num * 128) / nk;
    return (uint32_t)s;  // index = s >> 8, fraction = s & 255
}

__device__ void resize_tile(const uint8_t* __restrict__ src, int sw, int sh, int spitch,
                            uint8_t* __restrict__ dst, int w, int h, int pitch, int ty, int tx) {
    __shared__ uint32_t xs[RS_TX];
    __shared__ uint32_t ys[RS_TY];
    const int t = threadIdx.x;
    const int x_base = tx * RS_TX;
    const int y_base = ty * RS_TY;
    if (x_base + t < w) xs[t] = q8_coord(x_base + t, sw, w);
    if (t < RS_TY && y_base + t < h) ys[t] = q8_coord(y_base + t, sh, h);
    __syncthreads();

    const int lane = t & 63;
    const int wave = t >> 6;
    const int x0 = x_base + 4 * lane;
    if (x0 >= w) return;
    for (int r = wave; r < RS_TY; r += 4) {
        const int y = y_base + r;
        if (y >= h) break;
        const uint32_t sy = ys[r];
        const int ya = (int)(sy >> 8);
        const int fy = (int)(sy & 255);
        const int yb = min(ya + 1, sh - 1);
        const uint8_t* ra = src + (size_t)ya * spitch;
        const uint8_t* rb = src + (size_t)yb * spitch;
        uint32_t packed = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int x = x0 + q;
            uint32_t v = 0;
            if (x < w) {
                const uint32_t sx = xs[4 * lane + q];
                const int xa = (int)(sx >> 8);
                const int fx = (int)(sx & 255);
                const int xb = min(xa + 1, sw - 1);
                const int p00 = ra[xa], p01 = ra[xb], p10 = rb[xa], p11 = rb[xb];
                const int acc = (256 - fx) * (256 - fy) * p00 + fx * (256 - fy) * p01 +
                                (256 - fx) * fy * p10 + fx * fy * p11 + (1 << 15);
                v = (uint32_t)(acc >> 16);
            }
            packed |= v << (8 * q);
        }
        // pitch is a multiple of 16 >= w, so the 4-byte store stays in the row
        *reinterpret_cast<uint32_t*>(dst + (size_t)y * pitch + x0) = packed;
    }
}

struct ResizeArgs {
    const uint8_t* src;
    uint8_t* dst;
    int32_t sw, sh, spitch, n;
    int32_t prefix[PD_MAX_LEVELS + 1];  // first tile of each level
    int32_t w[PD_MAX_LEVELS], h[PD_MAX_LEVELS], pitch[PD_MAX_LEVELS];
    int64_t off[PD_MAX_LEVELS];
};

__global__ void __launch_bounds__(256) resize_single_kernel(ResizeArgs a) {
    const int b = blockIdx.x;
    int k = 0;
    while (k + 1 < a.n && a.prefix[k + 1] <= b) ++k;
    const int local = b - a.prefix[k];
    const int ntx = (a.w[k] + RS_TX - 1) / RS_TX;
    resize_tile(a.src, a.sw, a.sh, a.spitch, a.dst + a.off[k], a.w[k], a.h[k], a.pitch[k],
                local / ntx, local % ntx);
}

__global__ void __launch_bounds__(256) resize_table_kernel(const LevelItem* __restrict__ items,
                                                           const Tile* __restrict__ tiles) {
    const Tile tl = tiles[blockIdx.x];
    const LevelItem& it = items[tl.item];
    resize_tile(it.src, it.src_w, it.src_h, it.src_pitch, it.pyr, it.w, it.h, it.pitch, tl.ty, tl.tx);
}

}  // namespace

hipError_t launch_resize_single(const LevelItem* items, int n_items, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    ResizeArgs a = {};
    a.src = items[0].src;
    a.dst = items[0].pyr;
    a.sw = items[0].src_w;
    a.sh = items[0].src_h;
    a.spitch = items[0].src_pitch;
    a.n = n_items;
    int total = 0;
    for (int k = 0; k < n_items; ++k) {
        a.prefix[k] = total;
        a.w[k] = items[k].w;
        a.h[k] = items[k].h;
        a.pitch[k] = items[k].pitch;
        a.off[k] = items[k].pyr - items[0].pyr;
        total += resize_tiles_x(items[k].w) * resize_tiles_y(items[k].h);
    }
    a.prefix[n_items] = total;
    resize_single_kernel<<<total, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_resize_table(const LevelItem* items, const Tile* tiles, int n_tiles, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    resize_table_kernel<<<n_tiles, 256, 0, s>>>(items, tiles);
    return hipGetLastError();
}

}  // namespace pd
