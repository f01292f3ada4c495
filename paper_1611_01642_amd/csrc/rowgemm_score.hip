// Window scoring of one linear SVM on BF16 MFMA (Section 4.4, Algorithm 6),
// with the model's row offsets as the GEMM columns.
//
// A window (i, j) scores s = sum_a P[i + a][j][a] with
//   P[y][j][a] = sum_{b, c} F[y][j + b][c] * W[a][b][c],
// HOG rows a = 0..14 (b < 7, c < 36) and LBP rows a = 0..15 (b < 8, c < 59).
// For one feature row y, P is a dense GEMM: rows = 16 windows j, K = the
// window's (b, c) run of that row (contiguous when the row is staged
// channel-innermost), columns = the 16 offsets a.  So every staged feature
// row is multiplied once with the whole model (the window-row formulation
// re-reads each feature row for every window row it covers), and all 16
// MFMA columns are useful.  The diagonal sums run in a 16-slot ring of
// window-row accumulators in LDS: at row y, column a belongs to window row
// y - a; window row y - 15 is complete after row y.
//
// Numerics: HOG features are BF16 and the HOG weights their BF16 part; LBP
// counts are exact and the LBP weights are hi + lo BF16 halves (two MFMAs per A
// fragment).  FP32 accumulation; fixed summation order.
//
// Tile: a workgroup of 4 waves owns 64 window columns of one level (16 per
// wave) and streams down all feature rows; a row's loads are issued two rows
// ahead, so they are in flight during two rows of MFMAs.
#include <type_traits>

#include "pd_internal.h"

namespace pd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int RG_COLS = 64;
constexpr int RG_HOG_T = 8;    // K chunks of 32 per HOG row: 7 * 36 = 252 -> 256
constexpr int RG_LBP_T = 15;   // 8 * 60 = 480 (59 bins padded to 60)
constexpr int RG_HOG_C = PD_HOG_BLOCK;
constexpr int RG_LBP_C = 60;
constexpr int RG_HOG_SR = RG_COLS + PD_WIN_BLOCKS_X - 1;  // 70 staged blocks
constexpr int RG_LBP_SR = RG_COLS + PD_WIN_CELLS_X - 1;   // 71 staged cells
constexpr int RG_HOG_ROW = (RG_HOG_SR * RG_HOG_C + 8 + 7) / 8 * 8;
constexpr int RG_LBP_ROW = (RG_LBP_SR * RG_LBP_C + 8 + 7) / 8 * 8;

// packed B fragments: [HOG hi: t 8][LBP hi: t 15][LBP lo: t 15], each
// [lane 64][8] bf16 (lane: column a = lane % 16, K group lane / 16)
constexpr int RG_FRAG = 64 * 8;
constexpr int RG_PACKED = (RG_HOG_T + 2 * RG_LBP_T) * RG_FRAG;

struct RowShared {
    __bf16 hog[2][RG_HOG_ROW];
    __bf16 lbp[2][RG_LBP_ROW];
    __bf16 blbp[RG_LBP_T * RG_FRAG];  // the LBP weights' lo fragments
    float ring[4][16][16];  // per wave: window-row slot x window column
};

__global__ void pack_rowgemm_kernel(const float* __restrict__ w, uint16_t* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= RG_PACKED) return;
    const int f = e / RG_FRAG, r = e - f * RG_FRAG;
    const int lane = r >> 3, kk = r & 7;
    const int a = lane & 15;
    float v = 0.0f;
    bool lo = false;
    if (f < RG_HOG_T) {
        const int k = 32 * f + 8 * (lane >> 4) + kk;
        const int b = k / RG_HOG_C, c = k % RG_HOG_C;
        if (a < PD_WIN_BLOCKS_Y && b < PD_WIN_BLOCKS_X) v = w[(a * PD_WIN_BLOCKS_X + b) * PD_HOG_BLOCK + c];
    } else {
        const int t = (f - RG_HOG_T) % RG_LBP_T;
        lo = f >= RG_HOG_T + RG_LBP_T;
        const int k = 32 * t + 8 * (lane >> 4) + kk;
        const int b = k / RG_LBP_C, c = k % RG_LBP_C;
        if (b < PD_WIN_CELLS_X && c < PD_LBP_BINS) v = w[PD_HOG_DIM + (a * PD_WIN_CELLS_X + b) * PD_LBP_BINS + c];
    }
    const uint16_t hi = f32_to_bf16(v);
    out[e] = lo ? f32_to_bf16(v - __uint_as_float((uint32_t)hi << 16)) : hi;
}

template <bool HOG>
struct RowRegs {
    static constexpr int SR = HOG ? RG_HOG_SR : RG_LBP_SR;
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
// the row's byte offset as a scalar), and soff[q], its byte offset in the
// staged row (LBP: that of the word's first column).  HOG elements past the
// last are clamped to it (same value, same place).  An LBP word is read from inside its
// plane row: where columns 4 d .. 4 d + 3 reach past the row's end, from the
// row's last four bytes, and shifted down by the difference (kept in the top
// byte of soff), so that its columns inside the row get their counts; the
// rest (past the level, feeding no stored window) get finite values.
template <bool HOG>
struct RowOffsets {
    uint32_t goff[RowRegs<HOG>::N], soff[RowRegs<HOG>::N];
};

template <bool HOG>
__device__ __forceinline__ void row_offsets(RowOffsets<HOG>& o, int j0, int hcols, int hrows) {
    constexpr int U = RowRegs<HOG>::UNITS, NC = RowRegs<HOG>::NC;
    constexpr int C = HOG ? RG_HOG_C : RG_LBP_C;
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
            // value; byte k of the word is column 4 d + k (its channel's slot
            // RG_LBP_C values further on), the last word's column 71 past the
            // staged row is skipped
            if (o.soff[q] & 0x80000000u) continue;
            const uint32_t so = o.soff[q] & 0xffffffu;
            const uint32_t w = r.v[q] >> (8u * ((o.soff[q] >> 24) & 3u));
            const uint32_t col0 = so / (2u * RG_LBP_C);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t b = (w >> (8 * k)) & 255u;
                if (k < 3 || col0 + 3 < (uint32_t)RG_LBP_SR)
                    *reinterpret_cast<uint16_t*>(d + so + k * 2 * RG_LBP_C) =
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

__device__ __forceinline__ void rowgemm_tile(const LevelItem& it, const uint16_t* __restrict__ packed, float bias,
                                             int tx, RowShared& sm) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int hc = it.hc, wc = it.wc, hb = hc - 1, wb = wc - 1;
    const int ny = it.ny, nx = it.nx;
    const int j0 = tx * RG_COLS;
    const int mrow = lane & 15, kg = lane >> 4;
    // a wave whose 16 window columns lie past the level (a level's last tile)
    // stages rows with the others but does no MFMA work
    const bool col_live = j0 + 16 * wave < nx;

    // B fragments: HOG and LBP hi in registers, LBP lo in LDS (shared by the
    // 4 waves)
    bf16x8 bh[RG_HOG_T], blh[RG_LBP_T];
    const u32x4* pk = reinterpret_cast<const u32x4*>(packed);
#pragma unroll
    for (int t = 0; t < RG_HOG_T; ++t) bh[t] = __builtin_bit_cast(bf16x8, pk[t * 64 + lane]);
#pragma unroll
    for (int t = 0; t < RG_LBP_T; ++t) blh[t] = __builtin_bit_cast(bf16x8, pk[(RG_HOG_T + t) * 64 + lane]);
    for (int e = threadIdx.x; e < RG_LBP_T * 64; e += 256)
        reinterpret_cast<u32x4*>(sm.blbp)[e] = pk[(RG_HOG_T + RG_LBP_T) * 64 + e];
    for (int e = threadIdx.x; e < 4 * 16 * 16; e += 256) (&sm.ring[0][0][0])[e] = 0.0f;
    // zero the staged rows once so every value an MFMA reads is finite
    for (int e = threadIdx.x; e < (int)(sizeof(sm.hog) + sizeof(sm.lbp)) / 4; e += 256)
        reinterpret_cast<uint32_t*>(&sm.hog[0][0])[e] = 0u;
    __syncthreads();
    RowOffsets<true> oh;
    RowOffsets<false> ol;
    row_offsets<true>(oh, j0, wb, hb);
    row_offsets<false>(ol, j0, wc, hc);
    const auto rh_src = planes_rsrc(it.hog16, (uint64_t)PD_HOG_BLOCK * hb * wb * 2);
    const auto rl_src = planes_rsrc(it.lbp, (uint64_t)PD_LBP_BINS * hc * wc);
    // row 0 into LDS; row 1 (stored after step 0) into registers
    RowRegs<true> rh2[2];
    RowRegs<false> rl2[2];
    load_row_fast<true>(rh2[0], oh, rh_src, 0, wb, hb);
    load_row_fast<false>(rl2[0], ol, rl_src, 0, wc, hc);
    store_row_fast<true>(rh2[0], oh, sm.hog[0]);
    store_row_fast<false>(rl2[0], ol, sm.lbp[0]);
    if (1 < hc) {
        if (1 < hb) load_row_fast<true>(rh2[0], oh, rh_src, 1, wb, hb);
        load_row_fast<false>(rl2[0], ol, rl_src, 1, wc, hc);
    }
    __syncthreads();

    float (*ring)[16] = sm.ring[wave];
    // Step y: MFMAs on staged row y.  The row it stores at its end (y + 1)
    // was loaded one step earlier, and it issues the loads of row y + 2: a
    // row's loads have two steps of MFMAs to arrive.
    auto step = [&](int y, RowRegs<true>& ch, RowRegs<false>& cl, RowRegs<true>& nh, RowRegs<false>& nl)
                    __attribute__((always_inline)) {
        const int cur = y & 1;
        // issued on every step (the row index is clamped), so the number of
        // loads in flight is the same on every path and the store of row
        // y + 1 below waits only for its own loads
        load_row_fast<true>(nh, oh, rh_src, y + 2, wb, hb);
        load_row_fast<false>(nl, ol, rl_src, y + 2, wc, hc);
        // four accumulators (HOG even and odd chunks, LBP hi, LBP lo), so
        // consecutive MFMAs do not wait on one another; summed in a fixed order
        f32x4 acc_h = {0.0f, 0.0f, 0.0f, 0.0f}, acc_h1 = acc_h, acc_lh = acc_h, acc_ll = acc_h;
        if (col_live && y < hb) {
            const __bf16* row = sm.hog[cur] + (16 * wave + mrow) * RG_HOG_C + 8 * kg;
#pragma unroll
            for (int t = 0; t < RG_HOG_T; t += 2) {
                acc_h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_frag(row + 32 * t), bh[t], acc_h, 0, 0, 0);
                acc_h1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_frag(row + 32 * t + 32), bh[t + 1], acc_h1, 0, 0, 0);
            }
        }
        if (col_live) {
            const __bf16* row = sm.lbp[cur] + (16 * wave + mrow) * RG_LBP_C + 8 * kg;
            const bf16x8* bl = reinterpret_cast<const bf16x8*>(sm.blbp);
#pragma unroll
            for (int t = 0; t < RG_LBP_T; ++t) {
                const bf16x8 av = a_frag(row + 32 * t);
                acc_lh = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, blh[t], acc_lh, 0, 0, 0);
                acc_ll = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bl[t * 64 + lane], acc_ll, 0, 0, 0);
            }
        }
        const f32x4 acc = ((acc_h + acc_h1) + acc_lh) + acc_ll;
        // acc[r] = P[y][window 4*kg + r][a = mrow] belongs to window row y - a
        {
            const int i = y - mrow;
            if (i >= 0 && i < ny) {
#pragma unroll
                for (int r = 0; r < 4; ++r) ring[i & 15][4 * kg + r] += acc[r];
            }
        }
        if (y >= PD_WIN_CELLS_Y - 1) {  // window row y - 15 is complete
            const int i = y - (PD_WIN_CELLS_Y - 1);
            if (lane < 16) {
                const float v = ring[i & 15][lane];
                ring[i & 15][lane] = 0.0f;
                const int j = j0 + 16 * wave + lane;
                if (i < ny && j < nx) gmem(it.scores)[(size_t)i * nx + j] = v + bias;
            }
        }
        if (y + 1 < hc) {
            if (y + 1 < hb) store_row_fast<true>(ch, oh, sm.hog[cur ^ 1]);
            store_row_fast<false>(cl, ol, sm.lbp[cur ^ 1]);
        }
        __syncthreads();
    };
    // two register sets for rows in flight, alternating (unrolled by two so
    // that each is a fixed set of registers)
    for (int y = 0; y < hc; y += 2) {
        step(y, rh2[0], rl2[0], rh2[1], rl2[1]);
        if (y + 1 < hc) step(y + 1, rh2[1], rl2[1], rh2[0], rl2[0]);
    }
}

__global__ void __launch_bounds__(256) rowgemm_single_kernel(LevelItem it, const uint16_t* __restrict__ packed,
                                                             const float* __restrict__ bias) {
    __shared__ RowShared sm;
    rowgemm_tile(it, packed, bias[0], blockIdx.x, sm);
}

// With LOOP a capped grid strides over the tile table (each tile ends on a
// barrier).
template <bool LOOP>
__global__ void __launch_bounds__(256) rowgemm_table_kernel(const LevelItem* __restrict__ items,
                                                            const Tile* __restrict__ tiles, int n_tiles,
                                                            const uint16_t* __restrict__ packed,
                                                            const float* __restrict__ bias) {
    __shared__ RowShared sm;
    if constexpr (LOOP) {
        for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
            const Tile tl = tiles[t];
            rowgemm_tile(items[tl.item], packed, bias[0], tl.tx, sm);
        }
    } else {
        const Tile tl = tiles[blockIdx.x];
        rowgemm_tile(items[tl.item], packed, bias[0], tl.tx, sm);
    }
}

}  // namespace

int64_t rowgemm_packed_elems() { return RG_PACKED; }

hipError_t launch_pack_rowgemm(const float* w, uint16_t* out, hipStream_t s) {
    pack_rowgemm_kernel<<<ceil_div(RG_PACKED, 256), 256, 0, s>>>(w, out);
    return hipGetLastError();
}

hipError_t launch_rowgemm_single(const LevelItem& it, const uint16_t* packed, const float* bias, hipStream_t s) {
    if (it.nx <= 0 || it.ny <= 0) return hipSuccess;
    rowgemm_single_kernel<<<ceil_div(it.nx, RG_COLS), 256, 0, s>>>(it, packed, bias);
    return hipGetLastError();
}

hipError_t launch_rowgemm_table(const LevelItem* items, const Tile* tiles, int n_tiles, const uint16_t* packed,
                                const float* bias, int grid, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    if (grid > 0 && grid < n_tiles)
        rowgemm_table_kernel<true><<<grid, 256, 0, s>>>(items, tiles, n_tiles, packed, bias);
    else
        rowgemm_table_kernel<false><<<n_tiles, 256, 0, s>>>(items, tiles, n_tiles, packed, bias);
    return hipGetLastError();
}

}  // namespace pd
