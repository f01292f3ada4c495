// Window scoring of up to 8 linear SVMs at once on BF16 MFMA with FP32
// accumulation (Section 4.4, Algorithm 6, recast as a GEMM).
//
// GEMM view: rows = windows, K = the 11332 features of a window, columns =
// models.  LBP features are exact small integers, so each model's FP32 LBP
// weight w is split into two BF16 numbers, hi = bf16(w) and lo = bf16(w - hi),
// and both become GEMM columns: the 16 columns of one
// v_mfma_f32_16x16x32_bf16 hold 8 models x {hi, lo}, and a model's score is
// column hi + column lo.  HOG features are BF16 and their weights keep the
// BF16 part only, so a HOG MFMA's 16 columns hold 8 models at two offsets,
// serving two window rows.
//
// The K range of a window splits by window row offset a (15 HOG block rows,
// 16 LBP cell rows).  For a fixed a, window (i, j) reads feature row i + a,
// columns j .. j+6 (HOG) or j .. j+7 (LBP); staged channel-innermost, that is
// one contiguous run of 7*36 (padded to 256) or 8*60 (LBP channels padded to
// 60) values, which the MFMA A operand reads directly.
//
// Tile: a workgroup of 4 waves owns window rows i0..i0+3 x window columns
// j0..j0+63 (4 MFMA row tiles of 16), and the waves split the K chunks
// (chunk t goes to wave t % 4): every wave accumulates all 16 (row tile,
// window row) pairs over its chunks, and the four partial sums meet in LDS
// once per tile, in a fixed order.  The feature rows i0 .. i0+3+A-1 stream
// through a two-slot LDS ring (each loaded from HBM and converted once; the
// next row's loads are in flight during the current row's MFMAs).  For
// feature row r a wave reads each of its A fragments once and multiplies it
// with the B fragments of the up to four offsets a = r - i that reach its
// window rows; the B fragments of an offset are loaded from L2 when the
// offset first appears (one step ahead) into a register ring of four
// offsets, so each serves the four row tiles.  Per MFMA that is a quarter of
// an A fragment from LDS and a quarter of a B fragment from L2.
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
constexpr int MF_HOG_P = PD_WIN_BLOCKS_Y + 1;     // HOG weight slices: offset pairs (a, a + 1), a = -1 .. 14
constexpr int MF_LBP_T = 15;                      // 8*60 = 480
constexpr int MF_HOG_SR = MF_COLS + PD_WIN_BLOCKS_X - 1;  // 70 staged blocks per row
constexpr int MF_LBP_SR = MF_COLS + PD_WIN_CELLS_X - 1;   // 71 staged cells per row
constexpr int MF_HOG_ROW = MF_HOG_SR * MF_HOG_C + 8;      // bf16 per staged row (+ zero tail)
constexpr int MF_LBP_ROW = MF_LBP_SR * MF_LBP_C + 8;
constexpr int MF_ROW_MAX = ((MF_LBP_ROW > MF_HOG_ROW ? MF_LBP_ROW : MF_HOG_ROW) + 7) / 8 * 8;  // 16-byte rows

// Two staged feature rows; at the end of a tile the same memory holds the
// waves' partial sums, [wave][row tile][window row][lane] x 4.
union MfmaShared {
    __bf16 ring[2][MF_ROW_MAX];
    f32x4 red[4][4][MF_ROWS][64];
};

__device__ __forceinline__ uint16_t f2bf(float f) { return f32_to_bf16(f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---- weight packing --------------------------------------------------------
// HOG: [p 16][t 8][n 16][32]; LBP: [a 16][t 15][n 16][32] bf16; K index
// k = 32 t + kk maps to (b, c) = (k / C, k % C) of the offset row.  LBP:
// column n < 8 is the hi part of model n, n >= 8 the lo part of model n - 8.
// HOG features are BF16, and the HOG weights carry their BF16 part only, so
// a HOG slice holds two offsets: p = a + 1 for the pair (a, a + 1), column
// n < 8 model n at offset a, n >= 8 model n - 8 at offset a + 1 (zero outside
// 0 .. 14): one MFMA then serves two window rows.
__global__ void pack_weights_kernel(const float* __restrict__ w, int n_models, uint16_t* __restrict__ out) {
    const int hog_n = MF_HOG_P * MF_HOG_T * 16 * 32;
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
            const int off = n < 8 ? a - 1 : a;  // a is the slice index p here
            if (b < PD_WIN_BLOCKS_X && off >= 0 && off < PD_WIN_BLOCKS_Y)
                v = w[(size_t)m * PD_FEATURE_DIM + (off * PD_WIN_BLOCKS_X + b) * PD_HOG_BLOCK + c];
        } else {
            const int b = k / MF_LBP_C, c = k % MF_LBP_C;
            if (b < PD_WIN_CELLS_X && c < PD_LBP_BINS)
                v = w[(size_t)m * PD_FEATURE_DIM + PD_HOG_DIM + (a * PD_WIN_CELLS_X + b) * PD_LBP_BINS + c];
        }
    }
    const uint16_t hi = f2bf(v);
    // LBP counts are exact, so LBP weights carry hi + lo
    out[e] = (is_hog || n < 8) ? hi : f2bf(v - bf2f(hi));
}

// ---- scoring -----------------------------------------------------------------
// Feature row y (clamped) of the tile, channel-innermost in LDS: the loads
// are issued into registers first (load_row_fast) and written to LDS after
// MFMAs (store_row_fast), so their latency is hidden.
template <bool HOG>
struct RowRegs {
    static constexpr int SR = HOG ? MF_HOG_SR : MF_LBP_SR;
    static constexpr int NC = HOG ? PD_HOG_BLOCK : PD_LBP_BINS;
    // per plane row, HOG: SR BF16 values; LBP: the SR count bytes as 4-byte
    // words (columns 4 d .. 4 d + 3)
    static constexpr int UNITS = HOG ? SR : (SR + 3) / 4;
    // LBP: elements in blocks of 8 channels x UNITS words x 8 (64 channel
    // slots, those past the 59th empty), the channel fastest within a block
    static constexpr int N = HOG ? (UNITS * NC + 255) / 256 : (UNITS * 64 + 255) / 256;
    // HOG: BF16 bits; LBP: four raw counts (converted when stored)
    std::conditional_t<HOG, uint16_t, uint32_t> v[N];
};

// The per-thread offsets are taken once per tile: goff[q], the
// element's byte offset in the planes without the row (raw buffer loads add
// the row's byte offset as a scalar), and soff[q], its byte offset in a ring
// slot (LBP: that of the word's first column).  HOG elements past the last
// are clamped to it (same value, same slot).  An LBP word is read from inside its
// plane row: where columns 4 d .. 4 d + 3 reach past the row's end, from
// the row's last four bytes, and shifted down by the difference (kept in the
// top byte of soff), so that its columns inside the row get their counts;
// the rest (past the level, feeding no stored window) get finite values.
template <bool HOG>
struct RowOffsets {
    uint32_t goff[RowRegs<HOG>::N], soff[RowRegs<HOG>::N];
};

template <bool HOG>
__device__ __forceinline__ void row_offsets(RowOffsets<HOG>& o, int j0, int hcols, int hrows) {
    constexpr int U = RowRegs<HOG>::UNITS, NC = RowRegs<HOG>::NC;
    constexpr int C = HOG ? MF_HOG_C : MF_LBP_C;
    const uint32_t plane = (uint32_t)hrows * (uint32_t)hcols;
#pragma unroll
    for (int q = 0; q < RowRegs<HOG>::N; ++q) {
        if constexpr (HOG) {
            const int e = min((int)threadIdx.x + 256 * q, U * NC - 1);
            const int c = e / U, col = e - (e / U) * U;
            o.goff[q] = ((uint32_t)c * plane + (uint32_t)min(j0 + col, hcols - 1)) * 2u;
            o.soff[q] = (uint32_t)(col * C + c) * 2u;
        } else {
            // lanes by 8 channels x 8 words: a wave's staging writes fall in
            // 32 banks (words 4 columns apart are 120 dwords apart, channels
            // 2 bytes), its loads in 8 plane rows of 32 contiguous bytes.
            // Slots past the last channel or element load channel 58's word
            // and store nothing (bit 31 of soff).
            const int g = (int)threadIdx.x + 256 * q;
            const int cl = g & 7, rest = g >> 3;
            const int uu = rest % U, cb = rest / U;
            const int cc = 8 * cb + cl;
            const bool valid = cc < NC && cb < 8;
            const int cs = min(cc, NC - 1), col4 = 4 * uu;
            // hcols >= 8 (a level holds at least one window)
            const int start = min(j0 + col4, hcols - 4);
            o.goff[q] = (uint32_t)cs * plane + (uint32_t)start;
            o.soff[q] = (uint32_t)(col4 * C + cs) * 2u | (uint32_t)min(j0 + col4 - start, 3) << 24 |
                        (valid ? 0u : 0x80000000u);
        }
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
        else r.v[q] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, o.goff[q], roff, 0);
    }
}

template <bool HOG>
__device__ __forceinline__ void store_row_fast(const RowRegs<HOG>& r, const RowOffsets<HOG>& o, __bf16* dst) {
    uint8_t* d = reinterpret_cast<uint8_t*>(dst);
#pragma unroll
    for (int q = 0; q < RowRegs<HOG>::N; ++q) {
        if constexpr (HOG) {
            *reinterpret_cast<uint16_t*>(d + o.soff[q]) = r.v[q];
        } else {
            // LBP counts <= 64 are exact in BF16: the top half of their FP32
            // value; byte k of the word is column 4 d + k (its channel's
            // slot MF_LBP_C values further on), the last word's column 71
            // past the staged row is skipped
            if (o.soff[q] & 0x80000000u) continue;
            const uint32_t so = o.soff[q] & 0xffffffu;
            const uint32_t w = r.v[q] >> (8u * ((o.soff[q] >> 24) & 3u));
            const uint32_t col0 = so / (2u * MF_LBP_C);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t b = (w >> (8 * k)) & 255u;
                if (k < 3 || col0 + 3 < (uint32_t)MF_LBP_SR)
                    *reinterpret_cast<uint16_t*>(d + so + k * 2 * MF_LBP_C) =
                        (uint16_t)(__float_as_uint((float)b) >> 16);
            }
        }
    }
}

__device__ __forceinline__ bf16x8 a_frag(const __bf16* p) {  // 8-byte aligned run of 8 bf16
    const uint2 lo = *reinterpret_cast<const uint2*>(p);
    const uint2 hi = *reinterpret_cast<const uint2*>(p + 4);
    const u32x4 v = {lo.x, lo.y, hi.x, hi.y};
    return __builtin_bit_cast(bf16x8, v);
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
    // acc[m][ii]: row tile m (window columns j0 + 16 m ..), window row i0 + ii
    f32x4 acc[4][MF_ROWS];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int ii = 0; ii < MF_ROWS; ++ii) acc[m][ii] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // zero the staged rows once: every value an MFMA reads is then finite
    for (int e = threadIdx.x; e < (int)(sizeof(sm.ring) / 4); e += 256) reinterpret_cast<uint32_t*>(&sm.ring[0][0])[e] = 0u;
    __syncthreads();

    auto phase = [&](auto hog_tag) __attribute__((always_inline)) {
        constexpr bool HOG = decltype(hog_tag)::value;
        constexpr int A = HOG ? PD_WIN_BLOCKS_Y : PD_WIN_CELLS_Y;  // offsets
        constexpr int T = HOG ? MF_HOG_T : MF_LBP_T;                // K chunks
        constexpr int C = HOG ? MF_HOG_C : MF_LBP_C;
        constexpr int NQ = (T + 3) / 4;                            // chunks per wave (t = wave + 4 q)
        constexpr int S = A + MF_ROWS - 1;                         // feature rows of the tile
        const int hrows = HOG ? hb : hc, hcols = HOG ? wb : wc;
        const uint16_t* wsrc = HOG ? wpk : wpk + MF_HOG_P * MF_HOG_T * 16 * 32;
        constexpr int NS = HOG ? MF_HOG_P : A;                     // weight slices
        RowOffsets<HOG> ro;
        row_offsets<HOG>(ro, j0, hcols, hrows);
        const auto rsrc = planes_rsrc(HOG ? (const void*)hog16 : (const void*)lbp,
                                      (uint64_t)RowRegs<HOG>::NC * hrows * hcols * (HOG ? 2 : 1));
        // B fragment of slice a (HOG: the pair (a - 1, a)), chunk wave + 4 q:
        // this lane's 8 bf16
        auto load_b = [&](int a, int q) -> bf16x8 {
            const int t = min(wave + 4 * q, T - 1);
            const uint16_t* p = wsrc + ((size_t)(a * T + t) * 16 + mrow) * 32 + 8 * kg;
            return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
        };
        // a row's loads are issued two steps before it is stored
        constexpr int PF = 2;
        RowRegs<HOG> rr[PF];
        load_row_fast<HOG>(rr[0], ro, rsrc, i0, hcols, hrows);
        store_row_fast<HOG>(rr[0], ro, sm.ring[0]);
        if constexpr (PF == 2) load_row_fast<HOG>(rr[1], ro, rsrc, i0 + 1, hcols, hrows);
        // ring of B fragments by offset a % 4; the offset of the next step is
        // loaded one step ahead into bn
        bf16x8 bq[4][NQ], bn[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) bn[q] = load_b(0, q);
        __syncthreads();
        // step s: feature row i0 + s (ring slot s & 1) against offsets s - ii
        // of window rows ii = 0..3 (those with 0 <= s - ii < A)
        auto step = [&](int s, auto slot_tag) __attribute__((always_inline)) {
            constexpr int U = decltype(slot_tag)::value;  // s % 4
            const bool more = s + 1 < S;
            // the next row's loads, issued on every step (the row index is
            // clamped), so the count of loads in flight is the same on every
            // path; the new offset's B fragments move into the ring, and the
            // next offset's are loaded
#pragma unroll
            for (int q = 0; q < NQ; ++q) bq[U][q] = bn[q];
            load_row_fast<HOG>(rr[PF == 2 ? (U & 1) : 0], ro, rsrc, i0 + s + PF, hcols, hrows);
#pragma unroll
            for (int q = 0; q < NQ; ++q) bn[q] = load_b(min(s + 1, NS - 1), q);
            const __bf16* row = sm.ring[s & 1] + mrow * C + 8 * kg;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int t = wave + 4 * q;
                if (NQ * 4 > T && t >= T) break;  // uniform: the last wave has one chunk fewer
                bf16x8 av[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) av[m] = a_frag(row + 16 * m * C + 32 * t);
                if constexpr (HOG) {
                    // pairs (window rows 3, 2) with slice s - 2 into acc[m][0]
                    // and (1, 0) with slice s into acc[m][1]
                    if (s >= 2) {  // uniform; s - 2 <= 15 always
                        const bf16x8 bf = bq[(U - 2) & 3][q];
#pragma unroll
                        for (int m = 0; m < 4; ++m)
                            acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bf, acc[m][0], 0, 0, 0);
                    }
                    if (s < MF_HOG_P) {
                        const bf16x8 bf = bq[U][q];
#pragma unroll
                        for (int m = 0; m < 4; ++m)
                            acc[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bf, acc[m][1], 0, 0, 0);
                    }
                } else {
#pragma unroll
                    for (int ii = MF_ROWS - 1; ii >= 0; --ii) {
                        const int a = s - ii;
                        if (a < 0 || a >= A) continue;  // uniform
                        const bf16x8 bf = bq[(U - ii) & 3][q];
#pragma unroll
                        for (int m = 0; m < 4; ++m)
                            acc[m][ii] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bf, acc[m][ii], 0, 0, 0);
                    }
                }
            }
            if (more) store_row_fast<HOG>(rr[PF == 2 ? ((U + 1) & 1) : 0], ro, sm.ring[(s + 1) & 1]);
            __syncthreads();
        };
        for (int s = 0; s < S; s += 4) {
            step(s, std::integral_constant<int, 0>());
            if (s + 1 < S) step(s + 1, std::integral_constant<int, 1>());
            if (s + 2 < S) step(s + 2, std::integral_constant<int, 2>());
            if (s + 3 < S) step(s + 3, std::integral_constant<int, 3>());
        }
    };
    if (FEAT & PD_FEAT_HOG) {
        phase(std::integral_constant<bool, true>());
        // the HOG pair sums into the per-row layout: window row ii's HOG
        // score of model n in column n (where the LBP hi part adds to it),
        // columns 8..15 cleared for the LBP lo part
        const bool low = (lane & 15) < 8;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const f32x4 p32 = acc[m][0], p10 = acc[m][1];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float r2 = __shfl_down(p32[r], 8, 16), r0 = __shfl_down(p10[r], 8, 16);
                acc[m][3][r] = low ? p32[r] : 0.0f;
                acc[m][2][r] = low ? r2 : 0.0f;
                acc[m][1][r] = low ? p10[r] : 0.0f;
                acc[m][0][r] = low ? r0 : 0.0f;
            }
        }
    }
    if (FEAT & PD_FEAT_LBP) phase(std::integral_constant<bool, false>());

    // the waves' partial sums meet in LDS (the rows are no longer read: the
    // last step ended on a barrier); wave w finishes window row i0 + w,
    // adding the four partials in wave order
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int ii = 0; ii < MF_ROWS; ++ii) sm.red[wave][m][ii][lane] = acc[m][ii];
    __syncthreads();
    const int i = i0 + wave;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        f32x4 v = sm.red[0][m][wave][lane];
#pragma unroll
        for (int w = 1; w < 4; ++w) v += sm.red[w][m][wave][lane];
        // D layout: lane holds column n = lane % 16 for window columns
        // 4 * (lane / 16) + r of the row tile; model n's score = column n +
        // column n + 8
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float hi = v[r];
            const float lo = __shfl_down(hi, 8, 16);
            const int n = lane & 15;
            const int j = j0 + 16 * m + 4 * (lane >> 4) + r;
            if (n < 8 && n < n_models && i < ny && j < nx)
                scores[((size_t)n * ny + i) * nx + j] = (hi + lo) + bias[n];
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
    return (int64_t)(MF_HOG_P * MF_HOG_T + PD_WIN_CELLS_Y * MF_LBP_T) * 16 * 32;
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
