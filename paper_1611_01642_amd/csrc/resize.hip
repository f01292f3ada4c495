// Pyramid resize (Section 4.1 step 2, Section 4.4): every level is resampled
// from the level-0 image with pixel-centre-aligned bilinear interpolation in
// Q8 fixed point, rounded half up.  All arithmetic is integer, so results are
// exact.  One workgroup writes a tile of 256 columns x 16..128 rows of one
// level; the Q8 coordinates of the tile's columns and rows are computed once
// per tile in LDS, and the source rectangle the tile reads is staged in LDS
// with coalesced word loads, whole rows per pass, so the four taps of every
// output pixel are LDS reads (tiles whose rectangle does not fit read the
// taps from global memory instead).
#include "pd_internal.h"

namespace pd {
namespace {

// Q8 source coordinate of output sample `x` along an axis of n0 -> nk
// samples: ((2x + 1) n0 - nk) * 128 / nk, the integer quotient truncated,
// split into index (s >> 8) and fraction (s & 255).  Taken in double: the
// numerator (|num| < 2^39) and divisor convert exactly, and a quotient that is
// not an integer lies at least 1 / nk from one, far more than the rounding of
// the division (below |num / nk| 2^-53), so truncating the rounded quotient
// gives the integer quotient.
__device__ inline uint32_t q8_coord(int x, int n0, int nk) {
    const int64_t num = ((int64_t)(2 * x + 1) * n0 - nk) * 128;
    return (uint32_t)(int64_t)__builtin_trunc((double)num / (double)nk);
}

constexpr int RS_BATCH = 8;  // loads in flight per thread while staging

typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

// Output rows y_base .. y_base + rows - 1 (rows <= RS_TY_MAX), columns
// tx * RS_TX .. + RS_TX - 1.
__device__ __forceinline__ void resize_tile(gptr<const uint8_t> __restrict__ src, int sw, int sh, int spitch,
                            gptr<uint8_t> __restrict__ dst, int w, int h, int pitch, int y_base, int rows, int tx) {
    __shared__ uint32_t xs[RS_TX];
    __shared__ uint32_t ys[RS_TY_MAX];
    // 4 bytes past the rectangle's room: a right tap one column past the
    // image's last one is read (and weighted 0) there
    __shared__ __attribute__((aligned(16))) uint8_t stage[RS_LDS + 4];
    const int t = threadIdx.x;
    const int x_base = tx * RS_TX;
    if (w == sw && h == sh) {
        // the level is the image itself (every Q8 coordinate is the pixel's
        // own index, fraction 0): a copy.  Lane: 4 output bytes from the two
        // aligned source words that hold them; the second word is loaded only
        // if it holds one of those bytes inside the row, so no load leaves the
        // image's pages.
        const int x0 = x_base + 4 * (t & 63);
        if (x0 >= w) return;
        const uint32_t keep = w - x0 >= 4 ? 0xffffffffu : (1u << (8 * (w - x0))) - 1u;
        for (int r = t >> 6; r < rows; r += 4) {
            const int y = y_base + r;
            if (y >= h) break;
            const auto a = src + (size_t)y * spitch + x0;
            const int mis = (int)(reinterpret_cast<uintptr_t>(a) & 3);
            const auto wp = reinterpret_cast<gptr<const uint32_t>>(a - mis);
            const uint32_t w0 = wp[0];
            const uint32_t w1 = mis > 0 && x0 + 4 - mis < w ? wp[1] : 0u;
            const uint32_t v = __builtin_amdgcn_alignbyte(w1, w0, (uint32_t)mis);
            // pitch is a multiple of 16 >= w, so the 4-byte store stays in the row
            *reinterpret_cast<gptr<uint32_t>>(dst + (size_t)y * pitch + x0) = v & keep;
        }
        return;
    }
    if (x_base + t < w) xs[t] = q8_coord(x_base + t, sw, w);
    if (t < rows && y_base + t < h) ys[t] = q8_coord(y_base + t, sh, h);
    __syncthreads();

    // source rectangle of the tile: rows sy0..sy1, columns sx0..sx1
    const int xe = min(x_base + RS_TX, w) - 1 - x_base, ye = min(y_base + rows, h) - 1 - y_base;
    const int sx0 = (int)(xs[0] >> 8), sx1 = min((int)(xs[xe] >> 8) + 1, sw - 1);
    const int sy0 = (int)(ys[0] >> 8), sy1 = min((int)(ys[ye] >> 8) + 1, sh - 1);
    const int nrow = sy1 - sy0 + 1;
    const int span_w = (sx1 - sx0 + 7) / 4;  // aligned words per row, whatever the row's alignment
    const bool staged = span_w <= 256 && nrow * span_w * 4 <= RS_LDS;  // uniform over the workgroup
    if (staged) {
        // coalesced aligned words, K whole rows per pass: thread t takes word
        // wd of rows r0, r0 + K, ...  Raw buffer loads from the image's first
        // aligned word, bounded by the aligned word that holds its last byte
        // (so no load leaves the image's pages); a word's offset steps from
        // row to row by one add, and past the bound a load returns 0 (those
        // words are past the rectangle and never read)
        const int K = 256 / span_w;
        const int r0 = t / span_w, wd = t - r0 * span_w;
        const uint8_t* s8 = (const uint8_t*)src;
        const uint32_t sa = (uint32_t)(reinterpret_cast<uintptr_t>(s8) & 3);
        const uint64_t img_bytes = (uint64_t)sa + (uint64_t)(sh - 1) * spitch + sw;
        const auto rsrc = planes_rsrc(s8 - sa, (img_bytes + 3) & ~3ull);
        if (r0 < K) {
            // unaligned byte offset (from the aligned base) of the rectangle's
            // first byte in row r, for r = rb + K k
            uint32_t u = sa + (uint32_t)(sy0 + r0) * (uint32_t)spitch + (uint32_t)sx0;
            const uint32_t du = (uint32_t)K * (uint32_t)spitch;
            uint32_t* st = reinterpret_cast<uint32_t*>(stage) + r0 * span_w + wd;
            const int dst = K * span_w;
            for (int rb = r0; rb < nrow; rb += K * RS_BATCH) {
                uint32_t v[RS_BATCH];
#pragma unroll
                for (int k = 0; k < RS_BATCH; ++k) {
                    v[k] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (u & ~3u) + 4u * (uint32_t)wd, 0, 0);
                    u += du;
                }
#pragma unroll
                for (int k = 0; k < RS_BATCH; ++k)
                    if (rb + K * k < nrow) st[k * dst] = v[k];
                st += RS_BATCH * dst;
            }
        }
        __syncthreads();
    }

    const int lane = t & 63;
    const int wave = t >> 6;
    const int x0 = x_base + 4 * lane;
    if (x0 >= w) return;
    // this lane's four columns, once per tile: taps and weights (a column past
    // the edge repeats the last one; its byte is masked off)
    int xa[4], xb[4], wx[4];
    uint32_t keep = 0u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t sx = xs[min(x0 + q, w - 1) - x_base];
        xa[q] = (int)(sx >> 8);
        wx[q] = (int)(sx & 255);
        xb[q] = min(xa[q] + 1, sw - 1);
        if (x0 + q < w) keep |= 255u << (8 * q);
    }
    if (staged) {
        // Per column, the taps of both source rows side by side as 16-bit
        // halves: (256 - fx) p0 + fx p1 for the two rows in one packed
        // multiply and one packed multiply-add (at most 256 * 255 per half),
        // then (256 - fy) top + fy bot + 2^15 as one dot product (below
        // 2^25): the same integers as the scalar form.  The right tap is
        // read at xa + 1 from the same address; where the image clamps it to
        // xa its weight is 0 instead (256 p0 either way).
        u16x2 wl[4], wr[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int f = xb[q] > xa[q] ? wx[q] : 0;
            wl[q] = (u16x2)(uint16_t)(256 - f);
            wr[q] = (u16x2)(uint16_t)f;
            xa[q] -= sx0;
        }
        for (int r = wave; r < rows; r += 4) {
            const int y = y_base + r;
            if (y >= h) break;
            // wave-uniform row terms
            const uint32_t sy = __builtin_amdgcn_readfirstlane(ys[r]);
            const int ya = (int)(sy >> 8);
            const int fy = (int)(sy & 255);
            const int yb = min(ya + 1, sh - 1);
            const int oa = (int)(reinterpret_cast<uintptr_t>(src + (size_t)ya * spitch + sx0) & 3);
            const int ob = (int)(reinterpret_cast<uintptr_t>(src + (size_t)yb * spitch + sx0) & 3);
            const uint8_t* ra = stage + (ya - sy0) * span_w * 4 + oa;
            const uint8_t* rb = stage + (yb - sy0) * span_w * 4 + ob;
            u16x2 fw;
            fw.x = (uint16_t)(256 - fy);
            fw.y = (uint16_t)fy;
            uint32_t d[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                u16x2 p0, p1;
                p0.x = ra[xa[q]];
                p0.y = rb[xa[q]];
                p1.x = ra[xa[q] + 1];
                p1.y = rb[xa[q] + 1];
                d[q] = __builtin_amdgcn_udot2(p0 * wl[q] + p1 * wr[q], fw, 1u << 15, false);
            }
            // the bytes at bits 16..23, one per column
            const uint32_t packed = __builtin_amdgcn_perm(d[1], d[0], 0x0c0c0602u) |
                                    __builtin_amdgcn_perm(d[3], d[2], 0x06020c0cu);
            // pitch is a multiple of 16 >= w, so the 4-byte store stays in the row
            *reinterpret_cast<gptr<uint32_t>>(dst + (size_t)y * pitch + x0) = packed & keep;
        }
        return;
    }
    // (256-fx)(256-fy) p00 + fx (256-fy) p01 + (256-fx) fy p10 + fx fy p11,
    // + 2^15, >> 16, grouped by row (the same integer)
    for (int r = wave; r < rows; r += 4) {
        const int y = y_base + r;
        if (y >= h) break;
        const uint32_t sy = ys[r];
        const int ya = (int)(sy >> 8);
        const int fy = (int)(sy & 255);
        const int yb = min(ya + 1, sh - 1);
        const auto ra = src + (size_t)ya * spitch, rb = src + (size_t)yb * spitch;
        uint32_t packed = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int top = (256 - wx[q]) * (int)ra[xa[q]] + wx[q] * (int)ra[xb[q]];
            const int bot = (256 - wx[q]) * (int)rb[xa[q]] + wx[q] * (int)rb[xb[q]];
            packed |= (uint32_t)(((256 - fy) * top + fy * bot + (1 << 15)) >> 16) << (8 * q);
        }
        // pitch is a multiple of 16 >= w, so the 4-byte store stays in the row
        *reinterpret_cast<gptr<uint32_t>>(dst + (size_t)y * pitch + x0) = packed & keep;
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
    resize_tile(gmem(a.src), a.sw, a.sh, a.spitch, gmem(a.dst) + a.off[k], a.w[k], a.h[k], a.pitch[k],
                (local / ntx) * RS_TY, RS_TY, local % ntx);
}

// Workgroups are dealt to the XCDs round-robin; each XCD takes a contiguous
// run of the table instead, so the levels of a frame, which all read the same
// source image, mostly share one XCD's L2.
__global__ void __launch_bounds__(256) resize_table_kernel(const LevelItem* __restrict__ items,
                                                           const Tile* __restrict__ tiles, int n_tiles) {
    const int run = (n_tiles + N_XCD - 1) / N_XCD;
    const int t = (int)(blockIdx.x % N_XCD) * run + (int)(blockIdx.x / N_XCD);
    if (t >= n_tiles) return;
    const Tile tl = tiles[t];
    const LevelItem& it = items[tl.item];
    // tile: first row in ty, row count in pad
    resize_tile(gmem(it.src), it.src_w, it.src_h, it.src_pitch, gmem(it.pyr), it.w, it.h, it.pitch, tl.ty, tl.pad,
                tl.tx);
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
    resize_table_kernel<<<N_XCD * ((n_tiles + N_XCD - 1) / N_XCD), 256, 0, s>>>(items, tiles, n_tiles);
    return hipGetLastError();
}

}  // namespace pd
