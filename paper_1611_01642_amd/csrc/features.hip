// Feature extraction of one pyramid level: uniform-LBP cell histograms
// (Section 4.2, Algorithms 1-2) and L2-Hys-normalised HOG block histograms
// (Section 4.3, Algorithms 4-5) from a single pass over the pixels.
//
// Mapping: one wave64 owns a strip of 64 cell columns (one lane per 8x8 cell)
// and walks down a chunk of block rows.  For each cell row, a lane reads its cell's
// 10x10 pixel neighbourhood straight from global memory (one 8-byte load per
// pixel row, plus the two halo bytes; neighbouring lanes read neighbouring
// bytes, so the loads are coalesced) and processes its 64 pixels:
//   * LBP: 3x3 code -> uniform bin -> +1 on a byte counter in a lane-private
//     LDS word (an LDS add; no other lane touches these words);
//   * HOG: gradient -> magnitude and orientation -> votes into the cell's
//     "direction partials" A[dir][bin], where dir is the neighbouring cell
//     (3x3) whose centre the bilinear spatial weight points at.  A pixel's
//     linear orientation interpolation touches two bins, b and b + 1, and its
//     spatial weights two target columns and two target rows: eight
//     read-add-writes of lane-private LDS accumulators addressed by b, with
//     the weights taken as products of the separable factors.  After each half cell row the
//     accumulators of a finished target row are read into registers.
// A 16x16-pixel block's trilinear histogram (Algorithm 5) equals, for each of
// its four cell slots t, the sum over its four cells s of A[s][t - s]: votes
// towards cells outside the block are exactly the terms this sum leaves out,
// so every pixel is processed once although blocks overlap by 50 %.  The block
// of row by = cy - 1 is assembled when cell row cy is done, from the previous
// row's partials (kept in registers) and the current ones, with one-lane
// shuffles for the right-hand neighbour; then L2-Hys and planar stores
// (coalesced).  Strips overlap by one cell column, chunks by one cell row.
//
// Sums run in a fixed order, so results are bitwise reproducible.
#include "pd_internal.h"

namespace pd {
namespace {

__constant__ LbpTable kLbp = make_lbp_table();

// ---- atan in units of orientation bins ---------------------------------------
// atan(r) * 9 / pi for r in [0, 1] as r * P(r^2); coefficients fitted for this
// library (weighted least squares, see fit_atan.py); max error 4e-7 bins.
__device__ __forceinline__ float atan_bins(float r) {
    const float s = r * r;
    float p = -0.011615472845733166f;
    p = fmaf(p, s, 0.0626327395439148f);
    p = fmaf(p, s, -0.16017697751522064f);
    p = fmaf(p, s, 0.27622857689857483f);
    p = fmaf(p, s, -0.39845287799835205f);
    p = fmaf(p, s, 0.5714269876480103f);
    p = fmaf(p, s, -0.9548301696777344f);
    p = fmaf(p, s, 2.8647871017456055f);
    return p * r;
}

// Bilinear weight of pixel offset p in [0, 8) of a cell towards the centre of
// the neighbouring cell d in {-1, 0, 1}: 1 - |p + 0.5 - (8d + 4)| / 8, >= 0.
__host__ __device__ constexpr float sw(int p, int d) {
    const float dist = (float)p + 0.5f - (8.0f * (float)d + 4.0f);
    const float w = 1.0f - (dist < 0 ? -dist : dist) / 8.0f;
    return w > 0.0f ? w : 0.0f;
}

constexpr int LBP_WORDS = 15;  // 59 byte counters packed in words

// Orientation votes go to lane-private LDS accumulators [target cell
// row][dx + 1][bin] (bin 9 is bin 0 again, folded in when the accumulators are
// read), so a pixel adds to its two active bins at an address taken from its
// bin index instead of evaluating all nine.
constexpr int VOTE_BINS = PD_HOG_BINS + 1;
constexpr int VOTE_SLOTS = 2 * 3 * VOTE_BINS;

// What the previous cell row leaves for the next stays in registers, and the
// workgroup's LDS (lookup table, byte counters, vote accumulators: 76 KB)
// leaves room for two workgroups per CU.
struct FeatShared {
    uint32_t lut[256];                               // (increment << 7) | word
    uint32_t cnt[FT_WAVES][FT_W * LBP_WORDS];        // lane-private byte counters
    float vote[FT_WAVES][VOTE_SLOTS][FT_W];          // lane-private orientation votes
};

// One pixel row of a cell's neighbourhood: byte i (0..9) is pixel x0 - 1 + i.
struct PixRow {
    uint32_t lo, hi;   // own pixels x0..x0+7 (bytes 1..8)
    uint32_t halo;     // byte 0: pixel x0 - 1, byte 1: pixel x0 + 8 (clamped)
    uint32_t l0, l1;   // bytes 0..3 and 4..7: the left neighbours of lo, hi
    uint32_t r0, r1;   // bytes 2..5 and 6..9: the right neighbours of lo, hi
};

template <bool ALIGNED>
__device__ __forceinline__ PixRow load_row(gptr<const uint8_t> __restrict__ img, int pitch, int w, int y, int x0) {
    const auto p = img + (size_t)y * pitch + x0;
    PixRow r;
    if (ALIGNED) {
        const uint64_t m = *reinterpret_cast<gptr<const uint64_t>>(p);
        r.lo = (uint32_t)m;
        r.hi = (uint32_t)(m >> 32);
    } else {
        r.lo = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
        r.hi = (uint32_t)p[4] | ((uint32_t)p[5] << 8) | ((uint32_t)p[6] << 16) | ((uint32_t)p[7] << 24);
    }
    // the halo bytes (clamped at the image edges) from their own addresses, so
    // that no value depends on another load before it is used
    const auto row = img + (size_t)y * pitch;
    const uint32_t left = row[max(x0 - 1, 0)];
    const uint32_t right = row[min(x0 + 8, w - 1)];
    r.halo = left | (right << 8);
    r.l0 = __builtin_amdgcn_perm(r.lo, r.halo, 0x06050400u);
    r.l1 = __builtin_amdgcn_alignbyte(r.hi, r.lo, 3);
    r.r0 = __builtin_amdgcn_alignbyte(r.hi, r.lo, 1);
    r.r1 = __builtin_amdgcn_perm(r.halo, r.hi, 0x05030201u);
    return r;
}

// Per byte of four packed pixels, n >= c in bit 7 (the other bits are
// don't-care): the low seven bits are compared with the byte's top bit as a
// guard against borrows between bytes, and the top bits decide where they
// differ.
__device__ __forceinline__ uint32_t ge_bytes(uint32_t n, uint32_t c, uint32_t c_low) {
    const uint32_t d = (n | 0x80808080u) - c_low;
    // (n & ~c) | (~(n ^ c) & d) as one three-input bit operation
    return __builtin_amdgcn_bitop3_b32(n, c, d, 0xB2);
}

// Merges the eight comparison words (answer in bit 7 of each byte) into one
// LBP code per byte, neighbour k in bit 7 - k: the bit-reversed order of the
// code Algorithm 1 defines, which the lookup table below is built for.
__device__ __forceinline__ uint32_t lbp_codes4(const uint32_t (&r)[8]) {
    // (a & m) | (b & ~m) as one three-input bit operation
    auto sel = [](uint32_t m, uint32_t a, uint32_t b) { return __builtin_amdgcn_bitop3_b32(m, a, b, 0xCA); };
    const uint32_t t01 = sel(0x80808080u, r[0], r[1] >> 1), t23 = sel(0x80808080u, r[2], r[3] >> 1);
    const uint32_t t45 = sel(0x80808080u, r[4], r[5] >> 1), t67 = sel(0x80808080u, r[6], r[7] >> 1);
    const uint32_t q0 = sel(0xC0C0C0C0u, t01, t23 >> 2), q1 = sel(0xC0C0C0C0u, t45, t67 >> 2);
    return sel(0xF0F0F0F0u, q0, q1 >> 4);
}

__device__ __forceinline__ int px_at(const PixRow& r, int i) {  // i in 0..9, compile-time after unrolling
    if (i == 0) return (int)(r.halo & 255u);
    if (i == 9) return (int)((r.halo >> 8) & 255u);
    const int b = i - 1;
    return (int)(((b < 4 ? r.lo : r.hi) >> (8 * (b & 3))) & 255u);
}

// With CM the strip also emits the pruner's cell map: per cell, the 9-bin
// histogram with the full bilinear spatial kernel (every vote aimed at the
// cell: its own pixels' and its 8 neighbours', Sum_d A[c - d][d]), divided by
// sqrt(|h|^2 + eps^2), then the 59 LBP counts / 64: FP32 planar
// [68][hc][wc] (cmap) and/or BF16 channels-last [hc][wc][72] (cmap16).
// Lanes 1..62 own columns tx*62 .. tx*62 + 61, lanes 0 and 63 are halo, and
// the strip starts half a cell row early (the downward votes of the row
// above), so each owned cell sees all of its neighbours' partials.
template <int FEAT, bool ALIGNED, bool CM = false>
__device__ __forceinline__ void features_strip(gptr<const uint8_t> __restrict__ img, int w, int h, int pitch,
                                               gptr<float> __restrict__ hog, gptr<uint16_t> __restrict__ hog16,
                                               gptr<uint8_t> __restrict__ lbp, gptr<float> __restrict__ cmap,
                                               gptr<uint16_t> __restrict__ cmap16, int ty, int tx, int ch, float clip,
                                               float eps, FeatShared& sm, int wave, int group = 64) {
    constexpr bool DO_HOG = (FEAT & PD_FEAT_HOG) != 0;
    constexpr bool DO_LBP = (FEAT & PD_FEAT_LBP) != 0;
    static_assert(!CM || (DO_HOG && DO_LBP), "the cell map needs HOG and LBP");
    const int lane = threadIdx.x & 63;
    const int hc = h / PD_CELL, wc = w / PD_CELL;
    const int hb = hc - 1, wb = wc - 1;
    // lane groups (non-CM): a wave of `group`-lane groups, all on the same
    // columns, group g walking row chunk ty + g (narrow tail strips of a
    // level keep the wave's lanes busy); group = 64 is one strip
    const int li = CM ? lane : (lane & (group - 1));
    const int g = CM ? 0 : lane / group;
    const int cx0 = CM ? tx * FT_BX_CM : tx * FT_BX, cy0 = (ty + g) * ch;
    const int cx = CM ? cx0 - 1 + lane : cx0 + li;
    const int x0 = PD_CELL * min(max(cx, 0), wc - 1);  // lanes past the edges read valid pixels
    // a group past the level's last row chunk does nothing (empty row range)
    const int cy_last = cy0 <= max(hc - 2, 0) || cy0 == 0 ? min(cy0 + ch, hc - 1) : cy0 - 1;
    const int cy_start = (CM && cy0 > 0) ? cy0 - 1 : cy0;
    const bool own = !CM || (lane >= 1 && lane <= FT_BX_CM && cx < wc);
    const bool lbp_col = CM ? own : cx < wc && (li < group - 1 || cx == wc - 1);
    const bool blk_col = CM ? (own && cx < wb) : (li < group - 1 && cx < wb);
    const bool left_real = cx - 1 >= 0 && cx - 1 < wc, right_real = cx + 1 >= 0 && cx + 1 < wc;
    float down9[PD_HOG_BINS];  // CM: votes from the row above, gathered per target cell
#pragma unroll
    for (int k = 0; k < PD_HOG_BINS; ++k) down9[k] = 0.0f;
    // CM: the 9 votes aimed at this lane's cell from three source columns:
    // own (dx = 0), the right neighbour's dx = -1 and the left's dx = +1
    auto gather3 = [&](float l, float o, float r) -> float {
        const float fr = __shfl_down(l, 1, 64);
        const float fl = __shfl_up(r, 1, 64);
        return o + (right_real ? fr : 0.0f) + (left_real ? fl : 0.0f);
    };
    auto emit_cell = [&](int row, const float* hist) {
        float ss = 0.0f;
#pragma unroll
        for (int k = 0; k < PD_HOG_BINS; ++k) ss = fmaf(hist[k], hist[k], ss);
        const float inv = 1.0f / sqrtf(ss + eps * eps);
        if (own) {
            if (cmap) {
                const size_t plane = (size_t)hc * wc;
                const auto o = cmap + (size_t)row * wc + cx;
#pragma unroll
                for (int k = 0; k < PD_HOG_BINS; ++k) o[k * plane] = hist[k] * inv;
            }
            if (cmap16) {
                // a cell's 72 channels are 144 bytes, 16-byte aligned: channels
                // 0..7 in one 16-byte store, channel 8 in a 2-byte one
                const auto o = cmap16 + ((size_t)row * wc + cx) * PR_CP1;
                uint32_t h2[4];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    h2[k] = (uint32_t)f32_to_bf16(hist[2 * k] * inv) | ((uint32_t)f32_to_bf16(hist[2 * k + 1] * inv) << 16);
                *reinterpret_cast<gptr<uint4>>(o) = make_uint4(h2[0], h2[1], h2[2], h2[3]);
                o[8] = f32_to_bf16(hist[8] * inv);
            }
        }
    };
    // L2-Hys of one block (slots (r, c) in order (0,0), (0,1), (1,0), (1,1)),
    // stored into the planes at block row `row`, column cx
    auto store_block = [&](float (&v)[PD_HOG_BLOCK], int row) {
        const float e2 = eps * eps;
        float ss = 0.0f;
#pragma unroll
        for (int k = 0; k < PD_HOG_BLOCK; ++k) ss = fmaf(v[k], v[k], ss);
        float inv = 1.0f / sqrtf(ss + e2);
        float ss2 = 0.0f;
#pragma unroll
        for (int k = 0; k < PD_HOG_BLOCK; ++k) {
            v[k] = fminf(v[k] * inv, clip);
            ss2 = fmaf(v[k], v[k], ss2);
        }
        inv = 1.0f / sqrtf(ss2 + e2);
        const size_t plane = (size_t)hb * wb;
        const size_t at = (size_t)row * wb + cx;
        if (hog16) {  // BF16 planes (round to nearest even)
            auto o = hog16 + at;
#pragma unroll
            for (int k = 0; k < PD_HOG_BLOCK; ++k) {
                *o = f32_to_bf16(v[k] * inv);
                o += plane;
            }
        } else {
            auto o = hog + at;
#pragma unroll
            for (int k = 0; k < PD_HOG_BLOCK; ++k) {
                *o = v[k] * inv;
                o += plane;
            }
        }
    };
    uint32_t* cnt = &sm.cnt[wave][lane * LBP_WORDS];
    if (DO_LBP) {
#pragma unroll
        for (int k = 0; k < LBP_WORDS; ++k) cnt[k] = 0u;
    }
    // this lane's vote accumulators, [slot][lane] (slot stride FT_W words, so
    // the lanes of a wave hit distinct banks)
    float* vote = &sm.vote[wave][0][lane];
    if (DO_HOG) {
#pragma unroll
        for (int k = 0; k < VOTE_SLOTS; ++k) vote[k * FT_W] = 0.0f;
    }

    // In registers.  With CM, value (r*3 + c+1)*9 + k is the previous cell
    // row's partial of dir (dy = r, dx = c); after the top half of the next
    // row, r = 0 also holds that row's dy = -1 votes (the other term of the
    // same slots).  Without CM, value (r*2 + c)*9 + k is the sum aimed at slot
    // (r, c) of the block whose top-left cell is this lane's in the previous
    // row, from that row's two cells (and, after the top half of the next row,
    // from the next row's dy = -1 votes).
    float Pn[CM ? 6 * PD_HOG_BINS : 4 * PD_HOG_BINS];
    auto PV = [&](int i) -> float& { return Pn[i]; };
    // the two terms one cell row gives slot (r, c), c in {0, 1}, of the block
    // starting at this lane's column: own dx = c and the right lane's dx = c - 1
    auto pair = [&](const float (&X)[3][PD_HOG_BINS], int c, int k) -> float {
        return X[1 + c][k] + __shfl_down(X[c][k], 1, 64);
    };
    float Aa[3][PD_HOG_BINS], Ab[3][PD_HOG_BINS];  // [dx+1][bin] for two target rows
    // target row r's accumulators into X (bin 9 folded into bin 0), then
    // cleared for the next votes
    auto take = [&](int r, float (&X)[3][PD_HOG_BINS]) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float* q = vote + (r * 3 + a) * VOTE_BINS * FT_W;
#pragma unroll
            for (int k = 0; k < PD_HOG_BINS; ++k) X[a][k] = q[k * FT_W];
            X[a][0] += q[PD_HOG_BINS * FT_W];
#pragma unroll
            for (int k = 0; k < VOTE_BINS; ++k) q[k * FT_W] = 0.0f;
        }
    };

    // one pixel row: votes into Aa (upper target row) and Ab (lower target row)
    auto pixel_row = [&](int py, const PixRow& U, const PixRow& C, const PixRow& D, float s0, float s1,
                         bool count_lbp) {
        // LBP codes of the row's 8 pixels, four per word (Algorithm 1's
        // neighbours in its bit order: up-left, up, up-right, right,
        // down-right, down, down-left, left)
        uint32_t code4[2] = {0u, 0u};
        if (DO_LBP && count_lbp) {
            const uint32_t cw[2] = {C.lo, C.hi};
            const uint32_t nb[2][8] = {{U.l0, U.lo, U.r0, C.r0, D.r0, D.lo, D.l0, C.l0},
                                       {U.l1, U.hi, U.r1, C.r1, D.r1, D.hi, D.l1, C.l1}};
#pragma unroll
            for (int hw = 0; hw < 2; ++hw) {
                const uint32_t c_low = cw[hw] & 0x7f7f7f7fu;
                uint32_t r[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) r[k] = ge_bytes(nb[hw][k], cw[hw], c_low);
                code4[hw] = lbp_codes4(r);
            }
        }
#pragma unroll
        for (int px = 0; px < PD_CELL; ++px) {
            const int L = px_at(C, px), Rt = px_at(C, px + 2);
            const int T = px_at(U, px + 1), B = px_at(D, px + 1);
            if (DO_LBP && count_lbp) {
                const uint32_t e = sm.lut[(code4[px >> 2] >> (8 * (px & 3))) & 255u];
                // an LDS add: no read of the counter word comes back to the lane
                __hip_atomic_fetch_add(cnt + (e & 127u), e >> 7, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            if (DO_HOG) {
                // Algorithm 4, in FP32 from the start: the differences, their
                // squares and products are integers below 2^24, so every step
                // is exact, and |.| is a free source modifier
                const float dx = (float)(L - Rt);
                const float dy = (float)(T - B);
                const float ax = fabsf(dx), ay = fabsf(dy);
                const float mag = __builtin_amdgcn_sqrtf(fmaf(dy, dy, dx * dx));
                const float r = fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(fmaxf(ax, ay), 1.0f));
                const float u = atan_bins(r);  // [0, 2.25] bins
                // the angle in the first quadrant as 4.5 + e, e in [-4.5, 0]
                const float e = (ay > ax) ? -u : u - 4.5f;
                // folded to [0, 9] bins: 4.5 - e where dx and dy differ in sign
                // (e's sign bit flipped), else 4.5 + e; where one of them is
                // zero the two forms give the same votes (0 and 9 bins are one
                // orientation)
                const float ef = __uint_as_float(__float_as_uint(e) ^
                                                 ((__float_as_uint(dx) ^ __float_as_uint(dy)) & 0x80000000u));
                float t = 4.0f + ef;           // angle - 0.5: bin centres 10 + 20k degrees at integers
                t = t < 0.0f ? t + 9.0f : t;   // [0, 9]
                const int dxa = px < 4 ? -1 : 0;
                // linear interpolation between bins b and b + 1 (t = 9, a
                // rounding of t + 9 for tiny negative t, is bin 0: b = 8 gives
                // it all to slot 9, which is bin 0); the four trilinear
                // targets, target row tr (weight s0 or s1) by column dx (the
                // pixel's two bilinear column weights)
                const int b = min((int)t, PD_HOG_BINS - 1);
                const float wb = mag * (t - (float)b), wa = mag - wb;
                float* q = vote + b * FT_W;
#pragma unroll
                for (int tr = 0; tr < 2; ++tr)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const float k = sw(px, dxa + c) * (tr ? s1 : s0);
                        float* o = q + (tr * 3 + dxa + c + 1) * VOTE_BINS * FT_W;
                        // plain read-add-write: LDS float atomics run far slower
                        // than integer ones, and no other lane touches these words
                        o[0] += wa * k;
                        o[FT_W] += wb * k;
                    }
            }
        }
    };

    // The first cell row's three leading neighbourhood rows.  A cell row's
    // pixel loop ends holding the next cell row's (pixel rows 8 cy + 7 ..
    // 8 cy + 9, inside the image for every cell row but the last), so they
    // are loaded once per strip (clamped, so a lane group with no rows also
    // reads inside the image).
    PixRow U, C, D;
    {
        const int yb0 = PD_CELL * cy_start - 1 + ((CM && cy_start < cy0) ? 4 : 0);
        U = load_row<ALIGNED>(img, pitch, w, min(max(yb0, 0), h - 1), x0);
        C = load_row<ALIGNED>(img, pitch, w, min(yb0 + 1, h - 1), x0);
        D = load_row<ALIGNED>(img, pitch, w, min(yb0 + 2, h - 1), x0);
    }
    for (int cy = cy_start; cy <= cy_last; ++cy) {
        // CM's extra row above the strip: only its downward votes are needed
        const bool extra = CM && cy < cy0;
        const int yb = PD_CELL * cy - 1;  // pixel row of neighbourhood row 0
        float top[2][PD_HOG_BINS];  // CM: top slots of the blocks of row cy - 1
        if (DO_HOG) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int k = 0; k < PD_HOG_BINS; ++k) Aa[a][k] = Ab[a][k] = 0.0f;
        }
        // top half: pixel rows 0..3 vote towards cell rows -1 (Aa) and 0 (Ab)
        if (!extra) {
#pragma unroll 1
            for (int py = 0; py < 4; ++py) {
                const PixRow N = load_row<ALIGNED>(img, pitch, w, min(yb + py + 3, h - 1), x0);
                const float fpy = (float)py;
                pixel_row(py, U, C, D, (3.5f - fpy) * 0.125f, (4.5f + fpy) * 0.125f, true);
                U = C;
                C = D;
                D = N;
            }
        }
        if (DO_HOG) take(0, Aa);  // the top half's votes towards cell row -1
        if (DO_HOG) {
            if (cy > cy_start && !CM) {  // fold the dy = -1 votes into the top slots
#pragma unroll
                for (int k = 0; k < PD_HOG_BINS; ++k) {
                    PV(0 * 9 + k) += pair(Aa, 0, k);
                    PV(1 * 9 + k) += pair(Aa, 1, k);
                }
            }
            if (cy > cy_start && CM) {  // fold the dy = -1 votes into the previous row's r = 0 terms
                // the blocks' top slots first, summed as without CM
#pragma unroll
                for (int k = 0; k < PD_HOG_BINS; ++k) {
                    top[0][k] = (PV(1 * 9 + k) + __shfl_down(PV(0 * 9 + k), 1, 64)) + pair(Aa, 0, k);
                    top[1][k] = (PV(2 * 9 + k) + __shfl_down(PV(1 * 9 + k), 1, 64)) + pair(Aa, 1, k);
                }
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int k = 0; k < PD_HOG_BINS; ++k) PV(a * 9 + k) += Aa[a][k];
                {
                    // cell row cy - 1 is complete: votes from rows cy - 2 (down9),
                    // cy - 1 and cy (P r = 0); then row cy - 1's downward votes
                    float hist[PD_HOG_BINS];
#pragma unroll
                    for (int k = 0; k < PD_HOG_BINS; ++k)
                        hist[k] = down9[k] + gather3(PV(0 * 9 + k), PV(1 * 9 + k), PV(2 * 9 + k));
                    if (cy - 1 >= cy0) emit_cell(cy - 1, hist);
#pragma unroll
                    for (int k = 0; k < PD_HOG_BINS; ++k)
                        down9[k] = gather3(PV(3 * 9 + k), PV(4 * 9 + k), PV(5 * 9 + k));
                }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int k = 0; k < PD_HOG_BINS; ++k) Aa[a][k] = 0.0f;
        }
        // bottom half: pixel rows 4..7 vote towards cell rows +1 (Aa) and 0 (Ab)
#pragma unroll 1
        for (int py = 4; py < 8; ++py) {
            const PixRow N = load_row<ALIGNED>(img, pitch, w, min(yb + py + 3, h - 1), x0);
            const float fpy = (float)py;
            pixel_row(py, U, C, D, (fpy - 3.5f) * 0.125f, (11.5f - fpy) * 0.125f, !extra);
            U = C;
            C = D;
            D = N;
        }
        if (DO_HOG) {  // the bottom half's votes towards cell rows +1 and 0
            take(0, Aa);
            take(1, Ab);
        }

        // LBP histogram of this cell row
        if (DO_LBP) {
            const bool own_row = cy >= cy0 && (cy < cy0 + ch || cy == hc - 1);
            if (own_row && lbp_col) {
                const size_t plane = (size_t)hc * wc;
                auto o = lbp + (size_t)cy * wc + cx;
                // the 15 counter words once, then one byte store per bin
                uint32_t words[LBP_WORDS];
#pragma unroll
                for (int k = 0; k < LBP_WORDS; ++k) words[k] = cnt[k];
#pragma unroll
                for (int k = 0; k < PD_LBP_BINS; ++k, o += plane) *o = (uint8_t)(words[k >> 2] >> (8 * (k & 3)));
                if (CM && cmap) {
                    auto c = cmap + ((size_t)PD_HOG_BINS * hc + cy) * wc + cx;
#pragma unroll 1
                    for (int k = 0; k < PD_LBP_BINS; ++k, c += plane)
                        *c = (float)((cnt[k >> 2] >> (8 * (k & 3))) & 255u) * (1.0f / 64.0f);
                }
                if (CM && cmap16) {
                    // channels 9..71: counts / 64 (exact in BF16), then 4 zeros.
                    // Bytes 18..143 of the cell's 16-byte aligned record: a
                    // 2-, a 4- and an 8-byte store up to byte 32, then 7
                    // 16-byte stores
                    // A count is at most 64, so count / 64 has at most seven
                    // significant bits: exact in BF16, whose bits are then the
                    // FP32 value's upper half (no rounding step needed).
                    const auto cell = cmap16 + ((size_t)cy * wc + cx) * PR_CP1;
                    auto ch = [&](int c) -> float {  // channel c (9..71) as FP32
                        const int k = c - PD_HOG_BINS;
                        return k < PD_LBP_BINS ? (float)((cnt[k >> 2] >> (8 * (k & 3))) & 255u) * (1.0f / 64.0f)
                                               : 0.0f;
                    };
                    auto two = [&](int c) {  // BF16 bits of channels c, c + 1
                        return __builtin_amdgcn_perm(__float_as_uint(ch(c + 1)), __float_as_uint(ch(c)), 0x07060302u);
                    };
                    cell[9] = (uint16_t)(__float_as_uint(ch(9)) >> 16);
                    *reinterpret_cast<gptr<uint32_t>>(cell + 10) = two(10);
                    *reinterpret_cast<gptr<uint2>>(cell + 12) = make_uint2(two(12), two(14));
#pragma unroll 1
                    for (int c = 16; c < PR_CP1; c += 8)
                        *reinterpret_cast<gptr<uint4>>(cell + c) = make_uint4(two(c), two(c + 2), two(c + 4), two(c + 6));
                }
            }
#pragma unroll
            for (int k = 0; k < LBP_WORDS; ++k) cnt[k] = 0u;
        }

        if (DO_HOG) {
            // blocks of row cy - 1: top slots from P (CM: top), bottom slots the
            // previous row's terms + this row's terms S (which are also the next
            // row's top slots); both forms add the same terms in the same order
            float S[2][PD_HOG_BINS];
#pragma unroll
            for (int k = 0; k < PD_HOG_BINS; ++k) {
                S[0][k] = pair(Ab, 0, k);
                S[1][k] = pair(Ab, 1, k);
            }
            if (cy > cy0 && !CM) {
                float v[PD_HOG_BLOCK];
#pragma unroll
                for (int k = 0; k < PD_HOG_BINS; ++k) {
                    v[0 * 9 + k] = PV(0 * 9 + k);
                    v[1 * 9 + k] = PV(1 * 9 + k);
                    v[2 * 9 + k] = PV(2 * 9 + k) + S[0][k];
                    v[3 * 9 + k] = PV(3 * 9 + k) + S[1][k];
                }
                if (blk_col) store_block(v, cy - 1);
            }
            if (cy > cy0 && CM) {
                float v[PD_HOG_BLOCK];
#pragma unroll
                for (int k = 0; k < PD_HOG_BINS; ++k) {
                    v[0 * 9 + k] = top[0][k];
                    v[1 * 9 + k] = top[1][k];
                    v[2 * 9 + k] = (PV(4 * 9 + k) + __shfl_down(PV(3 * 9 + k), 1, 64)) + S[0][k];
                    v[3 * 9 + k] = (PV(5 * 9 + k) + __shfl_down(PV(4 * 9 + k), 1, 64)) + S[1][k];
                }
                if (blk_col) store_block(v, cy - 1);
            }
            if (cy < cy_last && !CM) {  // this row's slot sums for the next row's blocks
#pragma unroll
                for (int k = 0; k < PD_HOG_BINS; ++k) {
                    PV(0 * 9 + k) = S[0][k];
                    PV(1 * 9 + k) = S[1][k];
                    PV(2 * 9 + k) = pair(Aa, 0, k);
                    PV(3 * 9 + k) = pair(Aa, 1, k);
                }
            }
            if (cy < cy_last && CM) {  // this row's dy = 0 and dy = +1 partials become P
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int k = 0; k < PD_HOG_BINS; ++k) {
                        PV(a * 9 + k) = Ab[a][k];
                        PV((3 + a) * 9 + k) = Aa[a][k];
                    }
            }
        }
    }
    if (CM && cy_last == hc - 1) {  // the level's last cell row: no row below it
        float hist[PD_HOG_BINS];
#pragma unroll
        for (int k = 0; k < PD_HOG_BINS; ++k) hist[k] = down9[k] + gather3(Ab[0][k], Ab[1][k], Ab[2][k]);
        emit_cell(hc - 1, hist);
    }
}

// Indexed by the bit-reversed code that lbp_codes4 produces.
__device__ inline void init_lut(FeatShared& sm) {
    for (int c = threadIdx.x; c < 256; c += FT_WAVES * 64) {
        const int b = kLbp.bin[__brev(c) >> 24];
        sm.lut[c] = ((1u << (8 * (b & 3))) << 7) | (uint32_t)(b >> 2);
    }
}

template <int FEAT, bool ALIGNED>
__global__ void __launch_bounds__(FT_WAVES * 64) features_single_kernel(LevelItem it, float clip, float eps) {
    __shared__ FeatShared sm;
    init_lut(sm);
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int task = blockIdx.x * FT_WAVES + wave;
    const int ntx = feat_tiles_x(it.wc);
    if (task >= ntx * feat_tiles_y(it.hc)) return;
    features_strip<FEAT, ALIGNED>(gmem(it.pyr), it.w, it.h, it.pitch, gmem(it.hog), gmem(it.hog16), gmem(it.lbp),
                                  nullptr, nullptr, task / ntx, task % ntx, FT_CH, clip, eps, sm, wave);
}

template <bool ALIGNED>
__global__ void __launch_bounds__(FT_WAVES * 64) cellmap_single_kernel(LevelItem it, float clip, float eps) {
    __shared__ FeatShared sm;
    init_lut(sm);
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int task = blockIdx.x * FT_WAVES + wave;
    const int ntx = feat_tiles_x_cm(it.wc);
    if (task >= ntx * feat_tiles_y(it.hc)) return;
    features_strip<PD_FEAT_HOG | PD_FEAT_LBP, ALIGNED, true>(
        gmem(it.pyr), it.w, it.h, it.pitch, gmem(it.hog), gmem(it.hog16), gmem(it.lbp), gmem(it.cmap),
        gmem(it.cmap16), task / ntx, task % ntx, FT_CH, clip, eps, sm, wave);
}

__global__ void __launch_bounds__(FT_WAVES * 64) cellmap_table_kernel(const LevelItem* __restrict__ items,
                                                            const Tile* __restrict__ tiles, int n_tiles, int ch,
                                                            float clip, float eps) {
    __shared__ FeatShared sm;
    init_lut(sm);
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int task = blockIdx.x * FT_WAVES + wave; task < n_tiles; task += gridDim.x * FT_WAVES) {
        const Tile tl = tiles[task];
        const LevelItem& it = items[tl.item];
        features_strip<PD_FEAT_HOG | PD_FEAT_LBP, true, true>(gmem(it.pyr), it.w, it.h, it.pitch, gmem(it.hog),
                                                              gmem(it.hog16), gmem(it.lbp), gmem(it.cmap),
                                                              gmem(it.cmap16), tl.ty, tl.tx, ch, clip, eps, sm, wave);
    }
}

// The table launch requires 8-byte aligned level rows (pd_detect copies
// misaligned frames into the pyramid buffer).
template <int FEAT>
__global__ void __launch_bounds__(FT_WAVES * 64) features_table_kernel(const LevelItem* __restrict__ items,
                                                             const Tile* __restrict__ tiles, int n_tiles, int ch,
                                                             float clip, float eps) {
    __shared__ FeatShared sm;
    init_lut(sm);
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // strips are independent per wave; a capped grid loops over them
    for (int task = blockIdx.x * FT_WAVES + wave; task < n_tiles; task += gridDim.x * FT_WAVES) {
        const Tile tl = tiles[task];
        const LevelItem& it = items[tl.item];
        features_strip<FEAT, true>(gmem(it.pyr), it.w, it.h, it.pitch, gmem(it.hog), gmem(it.hog16), gmem(it.lbp),
                                   nullptr, nullptr, tl.ty, tl.tx, ch, clip, eps, sm, wave, tl.pad);
    }
}

// Algorithm 1 on its own: one thread per pixel (used to check the codes).
__global__ void __launch_bounds__(256) lbp_codes_kernel(const uint8_t* __restrict__ img, int w, int h,
                                                        int pitch, uint8_t* __restrict__ codes,
                                                        int codes_pitch) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= w || y >= h) return;
    auto at = [&](int yy, int xx) -> int {
        yy = min(max(yy, 0), h - 1);
        xx = min(max(xx, 0), w - 1);
        return img[(size_t)yy * pitch + xx];
    };
    const int c = at(y, x);
    const int code = (int)(at(y - 1, x - 1) >= c) | ((int)(at(y - 1, x) >= c) << 1) |
                     ((int)(at(y - 1, x + 1) >= c) << 2) | ((int)(at(y, x + 1) >= c) << 3) |
                     ((int)(at(y + 1, x + 1) >= c) << 4) | ((int)(at(y + 1, x) >= c) << 5) |
                     ((int)(at(y + 1, x - 1) >= c) << 6) | ((int)(at(y, x - 1) >= c) << 7);
    codes[(size_t)y * codes_pitch + x] = (uint8_t)code;
}

template <int FEAT, bool ALIGNED>
hipError_t feat_single(const LevelItem& it, float clip, float eps, hipStream_t s) {
    const int n = feat_tiles_x(it.wc) * feat_tiles_y(it.hc);
    features_single_kernel<FEAT, ALIGNED><<<ceil_div(n, FT_WAVES), FT_WAVES * 64, 0, s>>>(it, clip, eps);
    return hipGetLastError();
}

template <int FEAT>
hipError_t feat_single_any(const LevelItem& it, float clip, float eps, hipStream_t s) {
    const bool aligned = (((uintptr_t)it.pyr | (uintptr_t)it.pitch) & 7) == 0;
    return aligned ? feat_single<FEAT, true>(it, clip, eps, s) : feat_single<FEAT, false>(it, clip, eps, s);
}

template <int FEAT>
hipError_t feat_table(const LevelItem* items, const Tile* tiles, int n_tiles, float clip, float eps,
                      const Tuning& tu, hipStream_t s) {
    int blocks = ceil_div(n_tiles, FT_WAVES);
    if (tu.grid > 0) blocks = min(blocks, tu.grid);
    features_table_kernel<FEAT><<<blocks, FT_WAVES * 64, 0, s>>>(items, tiles, n_tiles, tu.feat_rows, clip, eps);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_features_cellmap_single(const LevelItem& it, float clip, float eps, hipStream_t s) {
    if (it.hc <= 0 || it.wc <= 0) return hipSuccess;
    const int n = feat_tiles_x_cm(it.wc) * feat_tiles_y(it.hc);
    const bool aligned = (((uintptr_t)it.pyr | (uintptr_t)it.pitch) & 7) == 0;
    if (aligned) cellmap_single_kernel<true><<<ceil_div(n, FT_WAVES), FT_WAVES * 64, 0, s>>>(it, clip, eps);
    else cellmap_single_kernel<false><<<ceil_div(n, FT_WAVES), FT_WAVES * 64, 0, s>>>(it, clip, eps);
    return hipGetLastError();
}

hipError_t launch_features_cellmap_table(const LevelItem* items, const Tile* tiles, int n_tiles, float clip,
                                         float eps, const Tuning& tu, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    int blocks = ceil_div(n_tiles, FT_WAVES);
    if (tu.grid > 0) blocks = min(blocks, tu.grid);
    cellmap_table_kernel<<<blocks, FT_WAVES * 64, 0, s>>>(items, tiles, n_tiles, tu.feat_rows, clip, eps);
    return hipGetLastError();
}

hipError_t launch_lbp_codes(const uint8_t* img, int w, int h, int pitch, uint8_t* codes, int codes_pitch,
                            hipStream_t s) {
    dim3 grid(ceil_div(w, 64), ceil_div(h, 4));
    lbp_codes_kernel<<<grid, 256, 0, s>>>(img, w, h, pitch, codes, codes_pitch);
    return hipGetLastError();
}

hipError_t launch_features_single(const LevelItem& it, int features, float clip, float eps, hipStream_t s) {
    if (it.hc <= 0 || it.wc <= 0) return hipSuccess;
    switch (features & (PD_FEAT_HOG | PD_FEAT_LBP)) {
        case PD_FEAT_HOG: return feat_single_any<PD_FEAT_HOG>(it, clip, eps, s);
        case PD_FEAT_LBP: return feat_single_any<PD_FEAT_LBP>(it, clip, eps, s);
        case PD_FEAT_HOG | PD_FEAT_LBP: return feat_single_any<PD_FEAT_HOG | PD_FEAT_LBP>(it, clip, eps, s);
        default: return hipSuccess;
    }
}

hipError_t launch_features_table(const LevelItem* items, const Tile* tiles, int n_tiles, int features,
                                 float clip, float eps, const Tuning& tu, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    switch (features & (PD_FEAT_HOG | PD_FEAT_LBP)) {
        case PD_FEAT_HOG: return feat_table<PD_FEAT_HOG>(items, tiles, n_tiles, clip, eps, tu, s);
        case PD_FEAT_LBP: return feat_table<PD_FEAT_LBP>(items, tiles, n_tiles, clip, eps, tu, s);
        case PD_FEAT_HOG | PD_FEAT_LBP:
            return feat_table<PD_FEAT_HOG | PD_FEAT_LBP>(items, tiles, n_tiles, clip, eps, tu, s);
        default: return hipSuccess;
    }
}

}  // namespace pd
