// Window scoring of up to 8 linear SVMs at once on BF16 MFMA with FP32
// accumulation (Section 4.4, Algorithm 6, recast as a GEMM).
//
// GEMM view: rows = windows, K = the 11332 features of a window, columns =
// models.  Each model's FP32 weight w is split into two BF16 numbers,
// hi = bf16(w) and lo = bf16(w - hi), and both become GEMM columns, so the 16
// columns of one v_mfma_f32_16x16x32_bf16 hold 8 models x {hi, lo}; a model's
// score is column hi + column lo.  LBP features are exact small integers, so
// their weights keep hi + lo (~16 bits); HOG features are BF16, and their
// weights keep the BF16 part only (the lo column is zero for HOG rows).
//
// The K range of a window splits by window row offset a (15 HOG block rows,
// 16 LBP cell rows).  For a fixed a, window (i, j) reads feature row i + a,
// columns j .. j+6 (HOG) or j .. j+7 (LBP); staged channel-innermost, that is
// one contiguous run of 7*36 (padded to 256) or 8*60 (LBP channels padded to
// 60) values, which the MFMA A operand reads directly.
//
// Tile: a workgroup of 4 waves owns window rows i0..i0+3 (one per wave) x
// window columns j0..j0+63 (4 MFMA row tiles of 16 per wave).  Loop over a:
// the 4 waves need feature rows i0+a .. i0+a+3, so rows pass through a 5-slot
// LDS ring (each row is loaded from HBM and converted once); the weight slice
// of offset a (packed B fragments) is staged once and shared by the 4 waves.
// A feature row's loads are issued two steps before it is stored (HBM
// latency spans two steps of MFMAs), a weight slice's one step before.
#include <type_traits>

#include "pd_internal.h"

namespace pd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int MF_COLS = 64;                       // window columns per tile
constexpr int MF_ROWS = 4;                        // window rows per tile (one per wave)
constexpr int MF_HOG_C = PD_HOG_BLOCK;            // 36 channels per block
constexpr int MF_LBP_C = 60;                      // 59 bins + 1 zero
constexpr int MF_HOG_T = 8;                       // K chunks of 32 per offset: 7*36 = 252 -> 256
constexpr int MF_LBP_T = 15;                      // 8*60 = 480
constexpr int MF_HOG_SR = MF_COLS + PD_WIN_BLOCKS_X - 1;  // 70 staged blocks per row
constexpr int MF_LBP_SR = MF_COLS + PD_WIN_CELLS_X - 1;   // 71 staged cells per row
constexpr int MF_HOG_ROW = MF_HOG_SR * MF_HOG_C + 8;      // bf16 per staged row (+ zero tail)
constexpr int MF_LBP_ROW = MF_LBP_SR * MF_LBP_C + 8;
constexpr int MF_RING = MF_ROWS + 1;
constexpr int MF_ROW_MAX = ((MF_LBP_ROW > MF_HOG_ROW ? MF_LBP_ROW : MF_HOG_ROW) + 7) / 8 * 8;  // 16-byte rows
constexpr int MF_B_ELEMS = MF_LBP_T * 16 * 32;            // packed B of one offset (LBP is larger)

struct MfmaShared {
    __bf16 ring[MF_RING][MF_ROW_MAX];
    __bf16 bw[2][MF_B_ELEMS];
};
static_assert((sizeof(__bf16) * MF_RING * MF_ROW_MAX) % 16 == 0, "weight slices must stay 16-byte aligned");

__device__ __forceinline__ uint16_t f2bf(float f) { return f32_to_bf16(f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---- weight packing --------------------------------------------------------
// HOG: [a 15][t 8][n 16][32]; LBP: [a 16][t 15][n 16][32] bf16.  Column n < 8
// is the hi part of model n, n >= 8 the lo part of model n - 8; K index
// k = 32 t + kk maps to (b, c) = (k / C, k % C) of the offset row.
__global__ void pack_weights_kernel(const float* __restrict__ w, int n_models, uint16_t* __restrict__ out) {
    const int hog_n = PD_WIN_BLOCKS_Y * MF_HOG_T * 16 * 32;
    const int lbp_n = PD_WIN_CELLS_Y * MF_LBP_T * 16 * 32;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= hog_n + lbp_n) return;
    const bool is_hog = e < hog_n;
    const int q = is_hog ? e : e - hog_n;
    const int T = is_hog ? MF_HOG_T : MF_LBP_T;
    const int kk = q & 31;
    const int n = (q >> 5) & 15;
    const int t = (q >> 9) % T;
    const int a = (q >> 9) / T;
    const int k = 32 * t + kk;
    const int m = n & 7;
    float v = 0.0f;
    if (m < n_models) {
        if (is_hog) {
            const int b = k / MF_HOG_C, c = k % MF_HOG_C;
            if (b < PD_WIN_BLOCKS_X) v = w[(size_t)m * PD_FEATURE_DIM + (a * PD_WIN_BLOCKS_X + b) * PD_HOG_BLOCK + c];
        } else {
            const int b = k / MF_LBP_C, c = k % MF_LBP_C;
            if (b < PD_WIN_CELLS_X && c < PD_LBP_BINS)
                v = w[(size_t)m * PD_FEATURE_DIM + PD_HOG_DIM + (a * PD_WIN_CELLS_X + b) * PD_LBP_BINS + c];
        }
    }
    const uint16_t hi = f2bf(v);
    // HOG features are BF16, so the HOG weights carry their BF16 part only;
    // LBP counts are exact, so LBP weights carry hi + lo
    out[e] = n < 8 ? hi : (is_hog ? (uint16_t)0 : f2bf(v - bf2f(hi)));
}

// ---- scoring -----------------------------------------------------------------
// Feature row y (clamped) of the tile, channel-innermost in LDS: the loads
// are issued into registers first (load_row_fast) and written to LDS after
// MFMAs (store_row_fast), so their latency is hidden.
template <bool HOG>
struct RowRegs {
    static constexpr int SR = HOG ? MF_HOG_SR : MF_LBP_SR;
    static constexpr int NC = HOG ? PD_HOG_BLOCK : PD_LBP_BINS;
    static constexpr int N = (SR * NC + 255) / 256;
    // HOG: BF16 bits; LBP: the raw count (converted when stored)
    std::conditional_t<HOG, uint16_t, uint32_t> v[N];
};

// The per-thread offsets are taken once per tile: goff[q], the
// element's byte offset in the planes without the row (raw buffer loads add
// the row's byte offset as a scalar), and soff[q], its byte offset in a ring
// slot.  Clamped elements repeat the last one (same value, same slot).
template <bool HOG>
struct RowOffsets {
    uint32_t goff[RowRegs<HOG>::N], soff[RowRegs<HOG>::N];
};

template <bool HOG>
__device__ __forceinline__ void row_offsets(RowOffsets<HOG>& o, int j0, int hcols, int hrows) {
    constexpr int SR = RowRegs<HOG>::SR, NC = RowRegs<HOG>::NC;
    constexpr int C = HOG ? MF_HOG_C : MF_LBP_C;
    const uint32_t plane = (uint32_t)hrows * (uint32_t)hcols;
#pragma unroll
    for (int q = 0; q < RowRegs<HOG>::N; ++q) {
        const int e = min((int)threadIdx.x + 256 * q, SR * NC - 1);
        const int c = e / SR, col = e - (e / SR) * SR;
        o.goff[q] = ((uint32_t)c * plane + (uint32_t)min(j0 + col, hcols - 1)) * (HOG ? 2u : 1u);
        o.soff[q] = (uint32_t)(col * C + c) * 2u;
    }
}

template <bool HOG>
__device__ __forceinline__ void load_row_fast(RowRegs<HOG>& r, const RowOffsets<HOG>& o, __amdgpu_buffer_rsrc_t rsrc,
                                              int y, int hcols, int hrows) {
    const uint32_t roff = (uint32_t)min(y, hrows - 1) * (uint32_t)hcols * (HOG ? 2u : 1u);
#pragma unroll
    for (int q = 0; q < RowRegs<HOG>::N; ++q) {
        // raw values: LBP counts are converted when stored, so that no
        // instruction waits on these loads before the MFMAs they overlap
        if (HOG) r.v[q] = __builtin_amdgcn_raw_buffer_load_b16(rsrc, o.goff[q], roff, 0);
        else r.v[q] = __builtin_amdgcn_raw_buffer_load_b8(rsrc, o.goff[q], roff, 0);
    }
}

template <bool HOG>
__device__ __forceinline__ void store_row_fast(const RowRegs<HOG>& r, const RowOffsets<HOG>& o, __bf16* dst) {
    uint8_t* d = reinterpret_cast<uint8_t*>(dst);
#pragma unroll
    for (int q = 0; q < RowRegs<HOG>::N; ++q) {
        // LBP counts <= 64 are exact in BF16: the top half of their FP32 value
        uint16_t v;
        if constexpr (HOG) v = r.v[q];
        else v = (uint16_t)(__float_as_uint((float)r.v[q]) >> 16);
        *reinterpret_cast<uint16_t*>(d + o.soff[q]) = v;
    }
}

template <int BSZ>
struct SliceRegs {
    static constexpr int N = (BSZ / 8 + 255) / 256;
    u32x4 v[N];
};

template <int BSZ>
__device__ __forceinline__ void load_slice(SliceRegs<BSZ>& r, const uint16_t* __restrict__ src) {
#pragma unroll
    for (int q = 0; q < SliceRegs<BSZ>::N; ++q) {
        const int e = min((int)threadIdx.x + 256 * q, BSZ / 8 - 1);
        r.v[q] = reinterpret_cast<const u32x4*>(src)[e];
    }
}

template <int BSZ>
__device__ __forceinline__ void store_slice(const SliceRegs<BSZ>& r, __bf16* dst) {
#pragma unroll
    for (int q = 0; q < SliceRegs<BSZ>::N; ++q) {
        const int e = threadIdx.x + 256 * q;
        if (e < BSZ / 8) reinterpret_cast<u32x4*>(dst)[e] = r.v[q];
    }
}

template <int FEAT>
__device__ __forceinline__ void mfma_tile(const uint16_t* __restrict__ hog16, const uint8_t* __restrict__ lbp,
                                          int wc, int hc, const uint16_t* __restrict__ wpk, const float* __restrict__ bias,
                                          int n_models, float* __restrict__ scores, int ty, int tx, MfmaShared& sm) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int hb = hc - 1, wb = wc - 1;
    const int ny = hc - PD_WIN_CELLS_Y + 1, nx = wc - PD_WIN_CELLS_X + 1;
    const int i0 = ty * MF_ROWS, j0 = tx * MF_COLS;
    const int mrow = lane & 15, kg = lane >> 4;
    f32x4 acc[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) acc[mt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // zero the LDS once: every value an MFMA reads is then finite
    for (int e = threadIdx.x; e < (int)(sizeof(MfmaShared) / 4); e += 256) reinterpret_cast<uint32_t*>(&sm)[e] = 0u;
    __syncthreads();

    auto phase = [&](auto hog_tag) __attribute__((always_inline)) {
        constexpr bool HOG = decltype(hog_tag)::value;
        constexpr int A = HOG ? PD_WIN_BLOCKS_Y : PD_WIN_CELLS_Y;
        constexpr int T = HOG ? MF_HOG_T : MF_LBP_T;
        constexpr int C = HOG ? MF_HOG_C : MF_LBP_C;
        constexpr int BSZ = T * 16 * 32;  // bf16 per offset slice
        const int hrows = HOG ? hb : hc, hcols = HOG ? wb : wc;
        const uint16_t* wsrc = HOG ? wpk : wpk + PD_WIN_BLOCKS_Y * MF_HOG_T * 16 * 32;
        // prologue: rows i0..i0+3 and the slice of offset 0 into LDS; row
        // i0+4 (stored after step 0) into registers
        RowOffsets<HOG> ro;
        row_offsets<HOG>(ro, j0, hcols, hrows);
        const auto rsrc = planes_rsrc(HOG ? (const void*)hog16 : (const void*)lbp,
                                      (uint64_t)RowRegs<HOG>::NC * hrows * hcols * (HOG ? 2 : 1));
        RowRegs<HOG> rows2[2];
        {
            for (int r = 0; r < MF_ROWS; ++r) {
                load_row_fast<HOG>(rows2[0], ro, rsrc, i0 + r, hcols, hrows);
                store_row_fast<HOG>(rows2[0], ro, sm.ring[r]);
            }
            SliceRegs<BSZ> sr;
            load_slice<BSZ>(sr, wsrc);
            store_slice<BSZ>(sr, sm.bw[0]);
            if (A > 1) load_row_fast<HOG>(rows2[0], ro, rsrc, i0 + MF_ROWS, hcols, hrows);
        }
        __syncthreads();
        // Step a: MFMAs on rows i0+a .. i0+a+3 with the slice of offset a.
        // The feature row it stores at its end (i0+a+4) was loaded one step
        // earlier, and it issues the load of row i0+a+5 for the next step: a
        // row's load has two steps of MFMAs to arrive.  The weight slice
        // (L2-resident) is loaded one step ahead.
        auto step = [&](int a, RowRegs<HOG>& cur, RowRegs<HOG>& nxt) __attribute__((always_inline)) {
            SliceRegs<BSZ> nsl;
            const bool more = a + 1 < A;
            // issued on every step (row and slice indices clamped), so the
            // number of loads in flight is the same on every path and the
            // stores below wait only for their own loads
            load_row_fast<HOG>(nxt, ro, rsrc, i0 + a + MF_ROWS + 1, hcols, hrows);
            load_slice<BSZ>(nsl, wsrc + (size_t)min(a + 1, A - 1) * BSZ);
            const __bf16* row = sm.ring[(a + wave) % MF_RING];
            const __bf16* bw = sm.bw[a & 1];
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const bf16x8 bf = *reinterpret_cast<const bf16x8*>(bw + (t * 16 + mrow) * 32 + 8 * kg);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    const __bf16* ap = row + (16 * mt + mrow) * C + 32 * t + 8 * kg;
                    const uint2 lo = *reinterpret_cast<const uint2*>(ap);
                    const uint2 hi = *reinterpret_cast<const uint2*>(ap + 4);
                    const u32x4 av = {lo.x, lo.y, hi.x, hi.y};
                    acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), bf, acc[mt], 0,
                                                                      0, 0);
                }
            }
            if (more) {  // slots not read in this step (see the ring indexing above)
                store_row_fast<HOG>(cur, ro, sm.ring[(a + MF_ROWS) % MF_RING]);
                store_slice<BSZ>(nsl, sm.bw[(a + 1) & 1]);
            }
            __syncthreads();
        };
        // two register sets for rows in flight, alternating (unrolled by two
        // so that each is a fixed set of registers)
        for (int a = 0; a < A; a += 2) {
            step(a, rows2[0], rows2[1]);
            if (a + 1 < A) step(a + 1, rows2[1], rows2[0]);
        }
    };
    if (FEAT & PD_FEAT_HOG) phase(std::integral_constant<bool, true>());
    if (FEAT & PD_FEAT_LBP) phase(std::integral_constant<bool, false>());

    // D layout: lane holds column n = lane % 16 for window rows 4*(lane/16) + r
    // of each 16-window tile; model n's score = column n + column n + 8.
    const int i = i0 + wave;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float v = acc[mt][r];
            const float lo = __shfl_down(v, 8, 16);
            const int n = lane & 15;
            const int j = j0 + 16 * mt + 4 * (lane >> 4) + r;
            if (n < 8 && n < n_models && i < ny && j < nx)
                scores[((size_t)n * ny + i) * nx + j] = (v + lo) + bias[n];
        }
    }
}

__global__ void __launch_bounds__(256) mfma_single_kernel(LevelItem it, const uint16_t* __restrict__ wpk,
                                                          const float* __restrict__ bias, int n_models, int feat) {
    __shared__ MfmaShared sm;
    const int ntx = ceil_div(it.nx, MF_COLS);
    const int ty = blockIdx.x / ntx, tx = blockIdx.x % ntx;
    if (feat == (PD_FEAT_HOG | PD_FEAT_LBP))
        mfma_tile<PD_FEAT_HOG | PD_FEAT_LBP>(it.hog16, it.lbp, it.wc, it.hc, wpk, bias, n_models, it.scores, ty, tx, sm);
    else if (feat == PD_FEAT_HOG)
        mfma_tile<PD_FEAT_HOG>(it.hog16, it.lbp, it.wc, it.hc, wpk, bias, n_models, it.scores, ty, tx, sm);
    else
        mfma_tile<PD_FEAT_LBP>(it.hog16, it.lbp, it.wc, it.hc, wpk, bias, n_models, it.scores, ty, tx, sm);
}

// With LOOP a capped grid strides over the tile table; the barrier at the end
// of each tile keeps the next tile's staging off LDS rows still being read.
template <bool LOOP>
__global__ void __launch_bounds__(256) mfma_table_kernel(const LevelItem* __restrict__ items,
                                                         const Tile* __restrict__ tiles, int n_tiles,
                                                         const uint16_t* __restrict__ wpk,
                                                         const float* __restrict__ bias, int n_models, int feat,
                                                         const int* __restrict__ n_dev) {
    __shared__ MfmaShared sm;
    if (n_dev) n_tiles = min(n_tiles, *n_dev);
    auto one = [&](int t) __attribute__((always_inline)) {
        const Tile tl = tiles[t];
        const LevelItem& it = items[tl.item];
        if (feat == (PD_FEAT_HOG | PD_FEAT_LBP))
            mfma_tile<PD_FEAT_HOG | PD_FEAT_LBP>(it.hog16, it.lbp, it.wc, it.hc, wpk, bias, n_models, it.scores,
                                                 tl.ty, tl.tx, sm);
        else if (feat == PD_FEAT_HOG)
            mfma_tile<PD_FEAT_HOG>(it.hog16, it.lbp, it.wc, it.hc, wpk, bias, n_models, it.scores, tl.ty, tl.tx, sm);
        else
            mfma_tile<PD_FEAT_LBP>(it.hog16, it.lbp, it.wc, it.hc, wpk, bias, n_models, it.scores, tl.ty, tl.tx, sm);
    };
    if constexpr (LOOP) {
        for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
            one(t);
            __syncthreads();
        }
    } else if ((int)blockIdx.x < n_tiles) {
        one(blockIdx.x);
    }
}

}  // namespace

int64_t packed_weight_elems() {
    return (int64_t)(PD_WIN_BLOCKS_Y * MF_HOG_T + PD_WIN_CELLS_Y * MF_LBP_T) * 16 * 32;
}

hipError_t launch_pack_weights(const float* w, int n_models, uint16_t* out, hipStream_t s) {
    const int n = (int)packed_weight_elems();
    pack_weights_kernel<<<ceil_div(n, 256), 256, 0, s>>>(w, n_models, out);
    return hipGetLastError();
}

hipError_t launch_mfma_single(const LevelItem& it, const uint16_t* wpk, const float* bias, int n_models, int features,
                              hipStream_t s) {
    if (it.nx <= 0 || it.ny <= 0) return hipSuccess;
    const int n = ceil_div(it.nx, MF_COLS) * ceil_div(it.ny, MF_ROWS);
    mfma_single_kernel<<<n, 256, 0, s>>>(it, wpk, bias, n_models, features & (PD_FEAT_HOG | PD_FEAT_LBP));
    return hipGetLastError();
}

hipError_t launch_mfma_table(const LevelItem* items, const Tile* tiles, int n_tiles, const uint16_t* wpk,
                             const float* bias, int n_models, int features, int grid, hipStream_t s,
                             const int* n_dev) {
    if (n_tiles <= 0) return hipSuccess;
    const int feat = features & (PD_FEAT_HOG | PD_FEAT_LBP);
    if (grid > 0 && grid < n_tiles)
        mfma_table_kernel<true><<<grid, 256, 0, s>>>(items, tiles, n_tiles, wpk, bias, n_models, feat, n_dev);
    else
        mfma_table_kernel<false><<<n_tiles, 256, 0, s>>>(items, tiles, n_tiles, wpk, bias, n_models, feat, n_dev);
    return hipGetLastError();
}

}  // namespace pd
