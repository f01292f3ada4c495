// Feature extraction of one pyramid level: uniform-LBP cell histograms
// (Section 4.2, Algorithms 1-2) and L2-Hys-normalised HOG block histograms
// (Section 4.3, Algorithms 4-5) from a single pass over the pixels.
//
// Mapping (one workgroup = 256 lanes = a tile of 16 x 16 cells; one lane per
// 8x8 cell):
//   1. the tile's pixels plus a one-pixel halo (130 x 130 bytes, clamped at
//      the image edge) are staged in LDS with coalesced 4-byte loads;
//   2. each lane walks the 64 pixels of its cell: LBP code -> uniform bin ->
//      one packed-byte LDS count; gradient -> magnitude and orientation ->
//      votes into its cell's 3x3 "direction partials" A[dir][bin], where dir
//      is the neighbouring cell whose centre the vote is weighted towards.
//      Each pixel votes into 2 cells x 2 cells x 2 bins;
//   3. a 16x16-pixel block's trilinear histogram (Algorithm 5: every pixel of
//      the block votes, bilinear in space towards the four cell centres of the
//      block, linear in orientation) equals, for each of its four cell slots
//      t, the sum over its four cells s of A[s][t - s].  Votes towards cells
//      outside the block are exactly the ones this sum leaves out.  So every
//      pixel is processed once instead of four times (blocks overlap 50 %);
//   4. L2-Hys per block and planar stores.
// The 16x16-cell tiles overlap by one cell so that all four cells of every
// block are inside one tile; a tile owns 15x15 blocks.
//
// Every LDS accumulator is owned by one lane, so sums run in a fixed order and
// results are bitwise reproducible.
#include "pd_internal.h"

namespace pd {
namespace {

// ---- uniform LBP table -------------------------------------------------------
// Codes with at most two circular 0/1 transitions take bins 0..57 in ascending
// code order; all others share bin 58.
struct LbpTable {
    uint8_t bin[256];
};

constexpr int popcount8(int v) {
    int n = 0;
    for (int k = 0; k < 8; ++k) n += (v >> k) & 1;
    return n;
}

constexpr LbpTable make_lbp_table() {
    LbpTable t{};
    int next = 0;
    for (int c = 0; c < 256; ++c) {
        const int rot = ((c >> 1) | (c << 7)) & 255;  // rotate right by one bit
        t.bin[c] = (uint8_t)(popcount8(c ^ rot) <= 2 ? next++ : 58);
    }
    return t;
}

__constant__ LbpTable kLbp = make_lbp_table();

// ---- atan in units of orientation bins ---------------------------------------
// atan(r) * 9 / pi for r in [0, 1] as r * P(r^2); coefficients fitted for this
// library (weighted least squares, see fit_atan.py); max error 4e-7 bins.
__device__ inline float atan_bins(float r) {
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

// ---- tile geometry -----------------------------------------------------------
constexpr int PX_SIDE = FT_C * PD_CELL;   // 128 pixels of whole cells
constexpr int PX_ROWS = PX_SIDE + 2;      // + halo row above and below
constexpr int PX_PITCH = 144;             // LDS column c <-> x = 8*cx0 - 8 + c
constexpr int PX_WORDS = PX_PITCH / 4;
constexpr int A_STRIDE = 81;              // 9 directions x 9 bins per cell
constexpr int L_STRIDE = 15;              // 59 byte counters packed in words

struct FeatSmem {
    uint8_t px[PX_ROWS * PX_PITCH];
    uint32_t lut[256];                    // (increment << 7) | word
    float A[FT_C * FT_C * A_STRIDE];
    uint32_t cnt[FT_C * FT_C * L_STRIDE];
};

// Bilinear weight of pixel offset p in [0, 8) of a cell towards the centre of
// the neighbouring cell d in {-1, 0, 1}: 1 - |p + 0.5 - (8d + 4)| / 8, >= 0.
__host__ __device__ constexpr float sw(int p, int d) {
    const float dist = (float)p + 0.5f - (8.0f * (float)d + 4.0f);
    const float w = 1.0f - (dist < 0 ? -dist : dist) / 8.0f;
    return w > 0.0f ? w : 0.0f;
}

template <int FEAT>
__device__ void features_tile(const uint8_t* __restrict__ img, int w, int h, int pitch,
                              float* __restrict__ hog, uint8_t* __restrict__ lbp, int ty, int tx,
                              float clip, float eps) {
    extern __shared__ __align__(16) uint8_t smem_raw[];
    FeatSmem& sm = *reinterpret_cast<FeatSmem*>(smem_raw);
    const int t = threadIdx.x;
    const int hc = h / PD_CELL, wc = w / PD_CELL;
    const int hb = hc - 1, wb = wc - 1;
    const int cy0 = ty * FT_B, cx0 = tx * FT_B;

    // 1. stage pixels (+ halo, clamped) and the LBP table
    const int y_org = cy0 * PD_CELL - 1;
    const int x_org = cx0 * PD_CELL - 8;
    const bool aligned = (((uintptr_t)img | (uintptr_t)pitch) & 3) == 0;
    for (int e = t; e < PX_ROWS * PX_WORDS; e += 256) {
        const int lr = e / PX_WORDS;
        const int q = e - lr * PX_WORDS;
        const int y = min(max(y_org + lr, 0), h - 1);
        const int x = x_org + 4 * q;
        const uint8_t* row = img + (size_t)y * pitch;
        uint32_t v;
        if (aligned && x >= 0 && x + 3 < w) {
            v = *reinterpret_cast<const uint32_t*>(row + x);
        } else {
            v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) v |= (uint32_t)row[min(max(x + b, 0), w - 1)] << (8 * b);
        }
        *reinterpret_cast<uint32_t*>(&sm.px[lr * PX_PITCH + 4 * q]) = v;
    }
    if (FEAT & PD_FEAT_LBP) {
        const int b = kLbp.bin[t];
        sm.lut[t] = ((1u << (8 * (b & 3))) << 7) | (uint32_t)(b >> 2);
    }
    const int cyl = t >> 4, cxl = t & 15;
    const int cy = cy0 + cyl, cx = cx0 + cxl;
    const bool cell_ok = cy < hc && cx < wc;
    float* Ac = &sm.A[t * A_STRIDE];
    uint32_t* Lc = &sm.cnt[t * L_STRIDE];
    if (FEAT & PD_FEAT_HOG) {
        for (int k = 0; k < A_STRIDE; ++k) Ac[k] = 0.0f;
    }
    if (FEAT & PD_FEAT_LBP) {
        for (int k = 0; k < L_STRIDE; ++k) Lc[k] = 0u;
    }
    __syncthreads();

    // 2. per-pixel work of this lane's cell
    if (cell_ok) {
        // row r (0..9) of the cell's 10x10 neighbourhood: bytes at LDS columns
        // 8*cxl + 7 .. 8*cxl + 16
        auto load_row = [&](int r, int (&v)[10]) {
            const uint8_t* p = &sm.px[(cyl * PD_CELL + r) * PX_PITCH + cxl * PD_CELL];
            const uint32_t a = *reinterpret_cast<const uint32_t*>(p + 4);
            const uint2 m = *reinterpret_cast<const uint2*>(p + 8);
            const uint32_t c = *reinterpret_cast<const uint32_t*>(p + 16);
            v[0] = (int)(a >> 24);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                v[1 + k] = (int)((m.x >> (8 * k)) & 255u);
                v[5 + k] = (int)((m.y >> (8 * k)) & 255u);
            }
            v[9] = (int)(c & 255u);
        };
        int ru[10], rm[10], rd[10];
        load_row(0, ru);
        load_row(1, rm);
#pragma unroll
        for (int py = 0; py < PD_CELL; ++py) {
            load_row(py + 2, rd);
#pragma unroll
            for (int px = 0; px < PD_CELL; ++px) {
                const int c = rm[px + 1];
                const int L = rm[px], R = rm[px + 2];
                const int T = ru[px + 1], B = rd[px + 1];
                if (FEAT & PD_FEAT_LBP) {
                    const int code = (int)(ru[px] >= c) | ((int)(T >= c) << 1) |
                                     ((int)(ru[px + 2] >= c) << 2) | ((int)(R >= c) << 3) |
                                     ((int)(rd[px + 2] >= c) << 4) | ((int)(B >= c) << 5) |
                                     ((int)(rd[px] >= c) << 6) | ((int)(L >= c) << 7);
                    const uint32_t e = sm.lut[code];
                    atomicAdd(&Lc[e & 127u], e >> 7);
                }
                if (FEAT & PD_FEAT_HOG) {
                    const int dx = L - R;       // Algorithm 4
                    const int dy = T - B;
                    const int ax = abs(dx), ay = abs(dy);
                    const int mn = min(ax, ay), mx = max(ax, ay);
                    const float mag = __builtin_amdgcn_sqrtf((float)(dx * dx + dy * dy));
                    const float r = (float)mn * __builtin_amdgcn_rcpf((float)max(mx, 1));
                    float u = atan_bins(r);                 // [0, 2.25] bins
                    u = (ay > ax) ? 4.5f - u : u;           // first quadrant
                    const float th = (dx * dy < 0) ? 9.0f - u : u;  // fold to [0, 180)
                    const float tb = th - 0.5f;             // bin centres at 10 + 20 k
                    const float fl = floorf(tb);
                    const float w1 = tb - fl;
                    int b0 = (int)fl;
                    b0 = b0 < 0 ? PD_HOG_BINS - 1 : min(b0, PD_HOG_BINS - 1);
                    const int b1 = b0 == PD_HOG_BINS - 1 ? 0 : b0 + 1;
                    const float v1 = mag * w1;
                    const float v0 = mag - v1;
                    const int dya = py < 4 ? -1 : 0;   // the two cell rows voted to
                    const int dxa = px < 4 ? -1 : 0;   // the two cell columns
#pragma unroll
                    for (int qy = 0; qy < 2; ++qy) {
#pragma unroll
                        for (int qx = 0; qx < 2; ++qx) {
                            const int ddy = dya + qy, ddx = dxa + qx;
                            const float s = sw(py, ddy) * sw(px, ddx);
                            const int dir = (ddy + 1) * 3 + (ddx + 1);
                            atomicAdd(&Ac[dir * PD_HOG_BINS + b0], v0 * s);
                            atomicAdd(&Ac[dir * PD_HOG_BINS + b1], v1 * s);
                        }
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                ru[k] = rm[k];
                rm[k] = rd[k];
            }
        }
    }
    __syncthreads();

    // 3a. LBP histograms of the cells this tile owns
    if (FEAT & PD_FEAT_LBP) {
        const int cy_end = (cy0 + FT_C >= hc) ? hc : cy0 + FT_B;
        const int cx_end = (cx0 + FT_C >= wc) ? wc : cx0 + FT_B;
        if (cell_ok && cy < cy_end && cx < cx_end) {
            const size_t plane = (size_t)hc * wc;
            uint8_t* o = lbp + (size_t)cy * wc + cx;
#pragma unroll
            for (int k = 0; k < PD_LBP_BINS; ++k)
                o[k * plane] = (uint8_t)((Lc[k >> 2] >> (8 * (k & 3))) & 255u);
        }
    }

    // 3b. HOG blocks: slot t of block (by, bx) sums A[s][t - s] over its cells s
    if (FEAT & PD_FEAT_HOG) {
        if (t < FT_B * FT_B) {
            const int byl = t / FT_B, bxl = t - (t / FT_B) * FT_B;
            const int by = cy0 + byl, bx = cx0 + bxl;
            if (by < hb && bx < wb) {
                float v[PD_HOG_BLOCK];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
#pragma unroll
                        for (int k = 0; k < PD_HOG_BINS; ++k) {
                            float acc = 0.0f;
#pragma unroll
                            for (int sy = 0; sy < 2; ++sy) {
#pragma unroll
                                for (int sx = 0; sx < 2; ++sx) {
                                    const int src = (byl + sy) * FT_C + (bxl + sx);
                                    const int dir = (r - sy + 1) * 3 + (c - sx + 1);
                                    acc += sm.A[src * A_STRIDE + dir * PD_HOG_BINS + k];
                                }
                            }
                            v[(r * 2 + c) * PD_HOG_BINS + k] = acc;
                        }
                    }
                }
                // 4. L2-Hys
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
                float* o = hog + (size_t)by * wb + bx;
#pragma unroll
                for (int k = 0; k < PD_HOG_BLOCK; ++k) o[k * plane] = v[k] * inv;
            }
        }
    }
}

constexpr size_t kFeatSmem = sizeof(FeatSmem);
static_assert(kFeatSmem <= 160 * 1024, "feature tile exceeds LDS");

template <int FEAT>
__global__ void __launch_bounds__(256) features_single_kernel(LevelItem it, float clip, float eps) {
    const int ntx = feat_tiles_x(it.wc);
    features_tile<FEAT>(it.pyr, it.w, it.h, it.pitch, it.hog, it.lbp, blockIdx.x / ntx,
                        blockIdx.x % ntx, clip, eps);
}

template <int FEAT>
__global__ void __launch_bounds__(256) features_table_kernel(const LevelItem* __restrict__ items,
                                                             const Tile* __restrict__ tiles,
                                                             float clip, float eps) {
    const Tile tl = tiles[blockIdx.x];
    const LevelItem& it = items[tl.item];
    features_tile<FEAT>(it.pyr, it.w, it.h, it.pitch, it.hog, it.lbp, tl.ty, tl.tx, clip, eps);
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

template <int FEAT>
hipError_t feat_single(const LevelItem& it, float clip, float eps, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&features_single_kernel<FEAT>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFeatSmem);
    if (attr != hipSuccess) return attr;
    const int n = feat_tiles_x(it.wc) * feat_tiles_y(it.hc);
    features_single_kernel<FEAT><<<n, 256, kFeatSmem, s>>>(it, clip, eps);
    return hipGetLastError();
}

template <int FEAT>
hipError_t feat_table(const LevelItem* items, const Tile* tiles, int n_tiles, float clip, float eps,
                      hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&features_table_kernel<FEAT>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFeatSmem);
    if (attr != hipSuccess) return attr;
    features_table_kernel<FEAT><<<n_tiles, 256, kFeatSmem, s>>>(items, tiles, clip, eps);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_lbp_codes(const uint8_t* img, int w, int h, int pitch, uint8_t* codes, int codes_pitch,
                            hipStream_t s) {
    dim3 grid(ceil_div(w, 64), ceil_div(h, 4));
    lbp_codes_kernel<<<grid, 256, 0, s>>>(img, w, h, pitch, codes, codes_pitch);
    return hipGetLastError();
}

hipError_t launch_features_single(const LevelItem& it, int features, float clip, float eps, hipStream_t s) {
    if (it.hc <= 0 || it.wc <= 0) return hipSuccess;
    switch (features & (PD_FEAT_HOG | PD_FEAT_LBP)) {
        case PD_FEAT_HOG: return feat_single<PD_FEAT_HOG>(it, clip, eps, s);
        case PD_FEAT_LBP: return feat_single<PD_FEAT_LBP>(it, clip, eps, s);
        case PD_FEAT_HOG | PD_FEAT_LBP: return feat_single<PD_FEAT_HOG | PD_FEAT_LBP>(it, clip, eps, s);
        default: return hipSuccess;
    }
}

hipError_t launch_features_table(const LevelItem* items, const Tile* tiles, int n_tiles, int features,
                                 float clip, float eps, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    switch (features & (PD_FEAT_HOG | PD_FEAT_LBP)) {
        case PD_FEAT_HOG: return feat_table<PD_FEAT_HOG>(items, tiles, n_tiles, clip, eps, s);
        case PD_FEAT_LBP: return feat_table<PD_FEAT_LBP>(items, tiles, n_tiles, clip, eps, s);
        case PD_FEAT_HOG | PD_FEAT_LBP:
            return feat_table<PD_FEAT_HOG | PD_FEAT_LBP>(items, tiles, n_tiles, clip, eps, s);
        default: return hipSuccess;
    }
}

}  // namespace pd
