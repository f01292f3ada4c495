// Window scoring in FP32 on the matrix cores (Section 4.4, Algorithm 6 recast
// as a GEMM on v_mfma_f32_16x16x4_f32: FP32 products, FP32 sums).
//
// The score of window (i, j) is the 2-D correlation
//   s(i, j) = sum_a sum_b sum_c F_c[i + a][j + b] * W[a][b][c] + bias.
// With one model a GEMM needs a second column dimension, and here it is the
// window's own column offsets: the 16 columns of an MFMA are 2 adjacent
// window rows x 8 column offsets.  For window rows (i, i + 1) and feature
// columns j0 .. j0 + 15,
//   O[m][(s, b)] = sum over feature rows r = i .. i + 16 and channels c of
//                  F_c[r][j0 + m] * W[r - i - s][b][c],
// with W zero outside the model's 15 HOG block rows / 16 LBP cell rows and,
// for HOG, past its 7 block columns: M = 16 feature columns, K = the pair's
// 16 (HOG) / 17 (LBP) feature rows x channels, in chunks of 4 channels of
// one row.  Window (i + s, j) then sums O[j + b - j0][(s, b)] over b = 0..7:
// a diagonal of the tile, begun in the tile to its left (a carry of 7
// windows per row).  The issued products are 1.13x the useful ones (the
// 17th / 16th row for the pair's second window row, HOG's eighth column
// offset) plus ragged tile and band edges; over the 1242x375 pyramid, 1.30x.
// (With the 16 row offsets as the columns instead, a feature row is
// multiplied with all 16 offsets, most of them outside the window grid near
// a level's top and bottom: 1.92x.)
//
// A workgroup of 8 waves owns a band of window rows of one level and walks
// a run of 64-column tiles left to right; wave (u, h) computes sub-tile u
// (feature columns 16 u .. 16 u + 15 of the tile) for the band's row pairs
// of parity h, so the waves' MFMA work per row differs by at most one pair.
// Each wave streams its sub-tile's feature rows through its own LDS region,
// with no barrier between waves: a row's 16 columns of all channels arrive
// as 16-byte loads (203 pieces, up to four per lane, two rows ahead in
// registers), are written channel-major, and read back as A fragments (one
// row, 4 channels, 16 columns: one 4-byte read per lane, no bank conflicts);
// the wave's LDS operations run in order, so the next row's writes follow
// the current row's reads.  The A fragments run against the B fragments of
// the wave's pairs that the row reaches, read from the model's weights in
// LDS (one 4-byte read per lane and MFMA).  The two waves of a sub-tile load
// the same rows, and the four sub-tiles of a tile share the rows' cache
// lines, close in time, so each feature row is fetched from memory about
// once per tile of a band (a band covers a whole level of a 1242x375
// frame).  A window's diagonal begins in the sub-tile to its left: at the
// end of a tile each wave hands its carry to the next through LDS (sub-tile
// 3's to sub-tile 0 of the next tile); a run that does not start its row
// first recomputes the tile to its left, in sub-tile 3 only.  Each window's
// sum runs in one order whatever the band, the run or the batch: per
// sub-tile, feature rows ascending, within a row the HOG then the LBP
// chunks; then the diagonal's b ascending within the window's sub-tile,
// plus the carry (b ascending within the sub-tile to its left), plus the
// bias.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "pd_internal.h"

namespace pd {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int S32_HOG_T = PD_HOG_BLOCK / 4;             // 9 chunks of 4 channels
constexpr int S32_LBP_T = (PD_LBP_BINS + 3) / 4;         // 15: channel 59 has zero weight
constexpr int S32_HOG_K = PD_WIN_BLOCKS_Y + 1;           // 16 feature rows per pair
constexpr int S32_LBP_K = PD_WIN_CELLS_Y + 1;            // 17
// Weight row a of the model (HOG 0 .. 14, LBP 0 .. 15) holds [t][b 8][c 4]
// floats, plus 2: the s = 1 lanes then read 2 banks away from the s = 0 ones.
// One zero row follows: the B fragments of rows a' - s outside the model
// read it.
constexpr int S32_HOG_RS = S32_HOG_T * 32 + 2;
constexpr int S32_LBP_RS = S32_LBP_T * 32 + 2;
constexpr int S32_HOG_N = PD_WIN_BLOCKS_Y * S32_HOG_RS;
constexpr int S32_LBP_N = PD_WIN_CELLS_Y * S32_LBP_RS;
constexpr int S32_ZERO = S32_HOG_N + S32_LBP_N;  // the zero row (S32_LBP_RS floats)
constexpr int S32_MODEL = (S32_ZERO + S32_LBP_RS + 3) / 4 * 4;  // floats per packed model (50 KB)
constexpr int S32_SUBS = 4;                              // sub-tiles per tile
constexpr int S32_WAVES = 2 * S32_SUBS;                  // waves per workgroup: sub-tile x pair parity
constexpr int S32_OS = 17;                               // row stride of a staged 16 x 16 O tile
constexpr int S32_SUB = 16;                              // feature columns per sub-tile (one MFMA's M)
constexpr int S32_TILE = S32_SUBS * S32_SUB;             // feature columns per tile
constexpr int S32_GRID_MAX = 512;                        // two workgroups per CU
// a wave's staged feature row (its sub-tile): HOG [36][16] floats, then LBP
// [60][16] bytes (channel 59 is never written: its weight is zero and any
// byte is finite); during a tile's write-back the same bytes hold the wave's
// O tile and its carries for the next sub-tile
constexpr int S32_STG_LBP = PD_HOG_BLOCK * S32_SUB * 4;
constexpr int S32_STAGE = S32_STG_LBP + 60 * S32_SUB;
constexpr int S32_PIECES_H = PD_HOG_BLOCK * S32_SUB / 4;  // 16-byte pieces of a staged row: 144 HOG
constexpr int S32_PIECES = S32_PIECES_H + PD_LBP_BINS;     // + 59 LBP
constexpr int S32_PPT = (S32_PIECES + 63) / 64;            // pieces per lane (4)

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ---- weight packing --------------------------------------------------------
// Model m's floats at m * S32_MODEL: HOG rows a = 0 .. 14, then LBP rows
// a = 0 .. 15, then the zero row; element (a, t, b, k) = W[a][b][4 t + k]
// (zero for HOG b = 7 and LBP channel 59).
__global__ void pack32_kernel(const float* __restrict__ w, int n_models, float* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_models * S32_MODEL) return;
    const int m = e / S32_MODEL, q = e - m * S32_MODEL;
    const float* wm = w + (size_t)m * PD_FEATURE_DIM;
    float v = 0.0f;
    if (q < S32_HOG_N) {
        const int a = q / S32_HOG_RS, x = q - a * S32_HOG_RS;
        const int t = x >> 5, b = (x >> 2) & 7, c = 4 * t + (x & 3);
        if (x < S32_HOG_T * 32 && b < PD_WIN_BLOCKS_X) v = wm[(a * PD_WIN_BLOCKS_X + b) * PD_HOG_BLOCK + c];
    } else if (q < S32_ZERO) {
        const int q2 = q - S32_HOG_N;
        const int a = q2 / S32_LBP_RS, x = q2 - a * S32_LBP_RS;
        const int t = x >> 5, b = (x >> 2) & 7, c = 4 * t + (x & 3);
        if (x < S32_LBP_T * 32 && c < PD_LBP_BINS) v = wm[PD_HOG_DIM + (a * PD_WIN_CELLS_X + b) * PD_LBP_BINS + c];
    }
    out[e] = v;
}

// ---- scoring -----------------------------------------------------------------
// Band table entry (Tile): item, ty = the band's first window row (even),
// tx = its run's first tile, pad = the run's tile count.  The table holds 8
// lists, one per XCD (entries xs.start[x] .. xs.start[x + 1] - 1, longest
// first); the workgroups on XCD x take its entries in turn from the counter
// ctr[model * 8 + x] (zero at launch).  NP: row pairs per band.
template <int FEAT, int NP>
__global__ void __launch_bounds__(64 * S32_WAVES) __attribute__((amdgpu_waves_per_eu(4)))
score32_kernel(const LevelItem* __restrict__ items, const Tile* __restrict__ bands, XcdLists xs,
               const float* __restrict__ packed, const float* __restrict__ bias, int* __restrict__ ctr,
               Decide32 dec) {
    constexpr bool HOG = (FEAT & PD_FEAT_HOG) != 0, LBP = (FEAT & PD_FEAT_LBP) != 0;
    constexpr int K = LBP ? S32_LBP_K : S32_HOG_K;  // feature rows per pair
    constexpr int NQ = NP / 2;                      // this wave's pairs: p = 2 q + h
    // write-back scratch in the wave's staging bytes: its O tile, then its
    // carries for the next sub-tile ([pair][row s][window 0..7] floats;
    // windows 8.. of a sub-tile lie within it)
    constexpr int O_FLOATS = 16 * S32_OS, C_FLOATS = NQ * 16;
    // decisions in this kernel: each wave keeps its NQ x 32 stored scores in
    // its O tile's bytes for them
    constexpr bool DEC = NQ * 32 <= O_FLOATS;
    static_assert((O_FLOATS + C_FLOATS) * 4 <= S32_STAGE, "write-back scratch");
    __shared__ float wsh[S32_MODEL];
    __shared__ __attribute__((aligned(16))) uint8_t stg[S32_WAVES][S32_STAGE];
    __shared__ float carry3[2][2][C_FLOATS];  // sub-tile 3's carry into the next tile, by tile parity and h
    __shared__ int item_k;
    // the decision terms of the current item (Decide32), read where the
    // scores are stored: no register holds them through the tile loop
    __shared__ struct {
        double thr;
        int32_t* count;  // NULL: no decisions here
        float* score;
        int4* key;
        int cap, level;
    } drec;
    const int model = blockIdx.y;
    {
        const float4* src = reinterpret_cast<const float4*>(packed + (size_t)model * S32_MODEL);
        float4* dst = reinterpret_cast<float4*>(wsh);
        for (int e = threadIdx.x; e < S32_MODEL / 4; e += 64 * S32_WAVES) dst[e] = src[e];
    }
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = wave / S32_SUBS;  // pair parity (the sub-tile rotates, below)
    const int col = lane & 15, kk = lane >> 4;  // A: feature column, channel within the chunk
    const int s = (lane >> 3) & 1, b = lane & 7;  // B: window row in the pair, column offset (kk: channel)
    // this lane's B element of weight row a' - s (a' = row within the pair's
    // K range), chunk 0; rows outside the model read the zero row
    const int blane = 4 * b + kk;
    auto b_hog = [&](int a) -> const float* {
        const int w = a - s;
        return wsh + ((unsigned)w < (unsigned)PD_WIN_BLOCKS_Y ? w * S32_HOG_RS : S32_ZERO) + blane;
    };
    auto b_lbp = [&](int a) -> const float* {
        const int w = a - s;
        return wsh + ((unsigned)w < (unsigned)PD_WIN_CELLS_Y ? S32_HOG_N + w * S32_LBP_RS : S32_ZERO) + blane;
    };
    uint8_t* const st = stg[wave];
    float* const ow = reinterpret_cast<float*>(st);
    float* const cw = ow + O_FLOATS;  // this wave's carries for the next sub-tile
    const float bm = bias[model];
    // write-back roles (lanes 0..31): window row e_s of the pair, window e_w
    // of the 16 the sub-tile completes (its columns - 7 .. + 8)
    const int e_s = (lane >> 4) & 1, e_w = lane & 15;
    const float* oe = ow + 8 * e_s;
    // this lane's pieces of a staged row: e = lane + 64 q, written at byte
    // 16 e; HOG (e < 144): channel e / 4, columns 4 (e % 4) ..; LBP: channel
    // e - 144 (the LBP bytes start at 16 * 144)
    static_assert(S32_STG_LBP == 16 * S32_PIECES_H, "pieces are laid out in order");
    auto is_h = [&](int q) { return HOG && lane + 64 * q < S32_PIECES_H; };
    auto is_l = [&](int q) { return LBP && lane + 64 * q >= S32_PIECES_H && lane + 64 * q < S32_PIECES; };
    const int x = blockIdx.x & 7;  // this workgroup's XCD (workgroups are dealt to the 8 XCDs in turn)
    const int first = xs.start[x], n_list = xs.start[x + 1] - first;
    int* const my_ctr = ctr + model * 8 + x;
    __syncthreads();

    for (;;) {
        if (tid == 0) item_k = __hip_atomic_fetch_add(my_ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int k = item_k;
        __syncthreads();
        if (k >= n_list) break;  // the whole workgroup, once the list is taken
        const Tile bt = bands[first + k];
        const LevelItem& it = items[bt.item];
        if (DEC && tid == 0) {
            drec.count = dec.counters ? dec.counters + it.frame : nullptr;
            if (dec.counters) {
                drec.thr = dec.thr[it.frame];
                drec.score = dec.cscore + it.cand_off;
                drec.key = dec.ckey + it.cand_off;
                drec.cap = it.cand_cap;
                drec.level = it.level;
            }
        }
        const int wc = it.wc, hc = it.hc, wb = wc - 1, hb = hc - 1, nx = it.nx, ny = it.ny;
        const int i0 = bt.ty;
        const int np = min(NP, (ny - i0 + 1) >> 1);  // pairs with a window row inside the level
        const int nrows = 2 * np + K - 2;
        const int n_sub = (wc + S32_SUB - 1) / S32_SUB;  // sub-tiles of the level's row
        const uint32_t hplane = (uint32_t)hb * (uint32_t)wb, lplane = (uint32_t)hc * (uint32_t)wc;
        const auto rh = planes_rsrc(it.hog, (uint64_t)PD_HOG_BLOCK * hplane * 4);
        // the buffer checks each dword of a load against its range: a 16-byte
        // LBP piece ending at the planes' end can start mid-dword, so the
        // range reaches 3 bytes further (into the level's own score buffer,
        // which follows its LBP planes) for that dword's valid bytes
        const auto rl = planes_rsrc(it.lbp, (uint64_t)PD_LBP_BINS * lplane + 3);
        const auto out = gmem(it.scores) + (size_t)model * ny * nx;
        const int tx_end = bt.tx + bt.pad;
        for (int tx = bt.tx > 0 ? bt.tx - 1 : 0; tx < tx_end; ++tx) {
            const bool lead = tx < bt.tx;  // only sub-tile 3's carry is wanted
            // this wave's sub-tile, rotated with the tile and the item: a
            // row's last tile holds fewer sub-tiles, and the waves of a
            // sub-tile share a SIMD, so a fixed mapping would leave the
            // same SIMDs idle on every row's last tile
            const int rot = (tx + k) & (S32_SUBS - 1);
            const int u = (wave + rot) & (S32_SUBS - 1);
            const int j0 = tx * S32_TILE + S32_SUB * u;  // this wave's first column
            // this wave computes when its sub-tile holds level columns and
            // it has pairs (uniform)
            const bool busy = S32_SUBS * tx + u < n_sub && h < np && (!lead || u == S32_SUBS - 1);
            f32x4 acc[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            if (busy) {
                // piece offsets without the row (a scalar): columns past the
                // level's edge read whatever finite values follow (they reach
                // only windows past the edge), and past the planes' end the
                // buffer returns zeros
                uint32_t voff[S32_PPT];
#pragma unroll
                for (int q = 0; q < S32_PPT; ++q) {
                    const int e = lane + 64 * q;
                    voff[q] = is_h(q) ? ((uint32_t)(e >> 2) * hplane + (uint32_t)(j0 + 4 * (e & 3))) * 4u
                                      : (uint32_t)max(e - S32_PIECES_H, 0) * lplane + (uint32_t)j0;
                }
                struct RowRegs {
                    u32x4 v[S32_PPT];
                };
                auto load = [&](int r, RowRegs& g) __attribute__((always_inline)) {
                    const uint32_t roh = (uint32_t)min(i0 + r, hb - 1) * (uint32_t)wb * 4u;
                    const uint32_t rol = (uint32_t)min(i0 + r, hc - 1) * (uint32_t)wc;
#pragma unroll
                    for (int q = 0; q < S32_PPT; ++q) {
                        if (is_h(q))
                            g.v[q] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rh, voff[q], roh, 0));
                        else if (is_l(q))
                            g.v[q] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rl, voff[q], rol, 0));
                    }
                };
                // row r: staged (after the previous row's reads, in the
                // wave's LDS order), read back as A fragments, against this
                // wave's pairs that reach it (K row a' = r - 2 p)
                auto row = [&](int r, RowRegs& g, int r_next) __attribute__((always_inline)) {
#pragma unroll
                    for (int q = 0; q < S32_PPT; ++q)
                        if (is_h(q) || is_l(q)) *reinterpret_cast<u32x4*>(st + 16 * (lane + 64 * q)) = g.v[q];
                    load(r_next, g);
                    __builtin_amdgcn_wave_barrier();
                    float ha[S32_HOG_T], lf[S32_LBP_T];
                    if constexpr (HOG) {
#pragma unroll
                        for (int t = 0; t < S32_HOG_T; ++t) ha[t] = reinterpret_cast<const float*>(st)[64 * t + lane];
                    }
                    if constexpr (LBP) {
#pragma unroll
                        for (int t = 0; t < S32_LBP_T; ++t) lf[t] = (float)st[S32_STG_LBP + 64 * t + lane];
                    }
                    __builtin_amdgcn_wave_barrier();
                    const int p_lo = max(0, (r - K + 2) >> 1), p_hi = min(np - 1, r >> 1);
                    // while it runs MFMA chains a wave issues ahead of the
                    // SIMD's waves that stage rows, keeping the MFMA pipe fed
                    __builtin_amdgcn_s_setprio(2);
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        const int p = 2 * q + h;
                        if (p < p_lo || p > p_hi) continue;  // uniform
                        const int a = r - 2 * p;
                        // the pair's B fragments (LDS reads the scheduler
                        // interleaves with the MFMAs; the other waves of the
                        // SIMD cover their latency)
                        constexpr int NH = HOG ? S32_HOG_T : 0, NB = NH + (LBP ? S32_LBP_T : 0);
                        float bv[NB];
                        if (!HOG || a < S32_HOG_K) {
#pragma unroll
                            for (int t = 0; t < NH; ++t) bv[t] = b_hog(a)[32 * t];
#pragma unroll
                            for (int t = NH; t < NB; ++t) bv[t] = b_lbp(a)[32 * (t - NH)];
#pragma unroll
                            for (int t = 0; t < NH; ++t)
                                acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ha[t], bv[t], acc[q], 0, 0, 0);
#pragma unroll
                            for (int t = NH; t < NB; ++t)
                                acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(lf[t - NH], bv[t], acc[q], 0, 0, 0);
                        } else if constexpr (LBP) {  // a = 16: the LBP rows only
#pragma unroll
                            for (int t = 0; t < S32_LBP_T; ++t) bv[t] = b_lbp(a)[32 * t];
#pragma unroll
                            for (int t = 0; t < S32_LBP_T; ++t)
                                acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(lf[t], bv[t], acc[q], 0, 0, 0);
                        }
                    }
                    __builtin_amdgcn_s_setprio(0);
                };
                // the next row's loads are issued as soon as this row is
                // staged, and are in flight during its MFMAs (issued on every
                // step: the row index is clamped)
                RowRegs g;
                load(0, g);
                for (int r = 0; r < nrows; ++r) row(r, g, r + 1);
            }
            // write-back.  1: per pair, the O tile through this wave's LDS;
            // lanes 0..31 sum their window's diagonal within the sub-tile
            // (b = 7 - e_w .. 7) and the carry for the next sub-tile's window
            // e_w (< 7: b = 0 .. 6 - e_w, columns 9 + e_w + b)
            float* const cnext = u == S32_SUBS - 1 ? carry3[tx & 1][h] : cw;
            float part[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                part[q] = 0.0f;
                if (2 * q + h >= np) continue;  // uniform
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int v = 0; v < 4; ++v) ow[(4 * kk + v) * S32_OS + col] = acc[q][v];
                __builtin_amdgcn_wave_barrier();
                if (lane < 32) {
                    float sum = 0.0f;
#pragma unroll
                    for (int bb = 0; bb < 8; ++bb) {
                        const int m = e_w - 7 + bb;
                        sum += m >= 0 ? oe[max(m, 0) * S32_OS + bb] : 0.0f;
                    }
                    float next = 0.0f;
#pragma unroll
                    for (int bb = 0; bb < 7; ++bb) {
                        const int m = 9 + e_w + bb;
                        next += m < 16 ? oe[min(m, 15) * S32_OS + bb] : 0.0f;
                    }
                    part[q] = sum;
                    if (e_w < 8) cnext[q * 16 + e_s * 8 + e_w] = next;
                }
            }
            __syncthreads();
            // 2: each window adds the carry from the sub-tile to its left
            // (sub-tile 0: sub-tile 3's of the previous tile, none at the
            // row's start)
            if (!lead && busy && lane < 32) {
                const int w_left = ((u - 1 - rot) & (S32_SUBS - 1)) + S32_SUBS * h;  // the wave of sub-tile u - 1
                const float* cin = u > 0 ? reinterpret_cast<const float*>(stg[w_left]) + O_FLOATS
                                         : (tx > 0 ? carry3[(tx - 1) & 1][h] : nullptr);
                const int jw = j0 - 7 + e_w;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int p = 2 * q + h;
                    if (p >= np) break;  // uniform
                    const float c = cin && e_w < 8 ? cin[q * 16 + e_s * 8 + e_w] : 0.0f;
                    const int i = i0 + 2 * p + e_s;
                    const bool in = jw >= 0 && jw < nx && i < ny;
                    const float v = (part[q] + c) + bm;
                    if (in) out[(size_t)i * nx + jw] = v;
                    if (DEC) ow[q * 32 + lane] = in ? v : __builtin_nanf("");  // the O tile is consumed
                }
                int32_t* const count = DEC ? drec.count : nullptr;
                if (count) {
                    // the decisions (Section 4.4), in a loop of their own: the
                    // wave's candidates take consecutive entries of the
                    // frame's list, one atomic per wave and pair
                    const double thr = drec.thr;
#pragma unroll 1
                    for (int q = 0; q < NQ; ++q) {
                        const int p = 2 * q + h;
                        if (p >= np) break;  // uniform
                        const float v = ow[q * 32 + lane];
                        const bool cand = (double)v > thr;  // false for NaN: no window
                        const uint64_t m = __ballot(cand);
                        if (!m) continue;
                        const int first_lane = __builtin_ctzll(m);
                        int base = 0;
                        if (lane == first_lane) base = atomicAdd(count, __popcll(m));
                        base = __shfl(base, first_lane, 64);
                        if (cand) {
                            const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
                            if (pos < drec.cap) {  // always: a window is appended once at most
                                drec.score[pos] = v;
                                drec.key[pos] = make_int4(drec.level, i0 + 2 * p + e_s, jw, 0);
                            }
                        }
                    }
                }
            }
            __syncthreads();  // the staging bytes are written again by the next tile
        }
    }
}

// row pairs per band for the tuning field's window rows per wave (4, 8, 16)
constexpr int s32_pairs(int rows) { return rows == 4 ? 8 : rows == 16 ? 24 : 16; }

template <int FEAT>
void launch_feat(int rows, dim3 grid, const LevelItem* items, const Tile* bands, const XcdLists& xs,
                 const float* packed, const float* bias, int* ctr, const Decide32& dec, hipStream_t s) {
    if (rows == 4)
        score32_kernel<FEAT, s32_pairs(4)><<<grid, 64 * S32_WAVES, 0, s>>>(items, bands, xs, packed, bias, ctr, dec);
    else if (rows == 16)
        score32_kernel<FEAT, s32_pairs(16)><<<grid, 64 * S32_WAVES, 0, s>>>(items, bands, xs, packed, bias, ctr, dec);
    else
        score32_kernel<FEAT, s32_pairs(8)><<<grid, 64 * S32_WAVES, 0, s>>>(items, bands, xs, packed, bias, ctr, dec);
}

}  // namespace

int64_t score32_packed_floats(int n_models) { return (int64_t)n_models * S32_MODEL; }

// Bands of 4 x `rows` window rows (`rows` = 4, 8 or 16 per wave) over runs
// of 16-column tiles, for every level of the table, as 8 lists, one per XCD,
// each longest first.  With 16 frames or more each frame's bands go to one
// XCD (frames dealt to the least loaded XCD, largest first), so the feature
// rows of neighbouring tiles and bands meet in one L2; with fewer, the bands
// themselves are dealt that way.  Runs: whole rows when the batch has enough
// bands for the machine, else runs of at least 2 tiles (each after the
// first recomputes one tile).  Returns the entry count; *grid is the launch
// width (a multiple of 8, at most two workgroups per CU).
int score32_bands(const LevelItem* items, int n_items, int rows, int grid_cap, Tile* out, XcdLists* xs,
                  int* grid) {
    const int P = s32_pairs(rows), band = 2 * P;
    int64_t n_whole = 0, tiles = 0;
    int n_frames = 0;
    for (int q = 0; q < n_items; ++q) {
        n_frames = std::max(n_frames, items[q].frame + 1);
        if (items[q].nx <= 0 || items[q].ny <= 0) continue;
        const int nb = ceil_div(items[q].ny, band);
        n_whole += nb;
        tiles += (int64_t)nb * ceil_div(items[q].wc, S32_TILE);  // 64-column tiles
    }
    const int run = n_whole >= 512 ? (1 << 30) : (int)std::max<int64_t>(2, (tiles + 1023) / 1024);
    struct Band {
        Tile t;
        int64_t cost;
    };
    std::vector<Band> all;
    std::vector<int64_t> frame_cost(n_frames, 0);
    for (int q = 0; q < n_items; ++q) {
        const LevelItem& it = items[q];
        if (it.nx <= 0 || it.ny <= 0) continue;
        const int nt = ceil_div(it.wc, S32_TILE);
        for (int i0 = 0; i0 < it.ny; i0 += band) {
            const int pairs = std::min(P, (it.ny - i0 + 1) / 2);
            for (int tx = 0; tx < nt; tx += run) {
                const int n = std::min(run, nt - tx);
                // the workgroup's row steps (barriers) over its tiles
                const int64_t cost = (int64_t)(n + (tx > 0)) * (2 * pairs + S32_LBP_K - 2);
                all.push_back(Band{Tile{q, i0, tx, n}, cost});
                frame_cost[it.frame] += cost;
            }
        }
    }
    auto by_cost = [](const Band& u, const Band& v) { return u.cost > v.cost; };
    std::vector<int> xcd_of;  // per frame (16 frames or more)
    int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    auto least = [&]() { return (int)(std::min_element(load, load + 8) - load); };
    if (n_frames >= 16) {
        std::vector<int> order(n_frames);
        for (int f = 0; f < n_frames; ++f) order[f] = f;
        std::stable_sort(order.begin(), order.end(), [&](int u, int v) { return frame_cost[u] > frame_cost[v]; });
        xcd_of.assign(n_frames, 0);
        for (int f : order) {
            const int x = least();
            xcd_of[f] = x;
            load[x] += frame_cost[f];
        }
    }
    std::stable_sort(all.begin(), all.end(), by_cost);
    std::vector<std::vector<Tile>> lists(8);
    for (const Band& u : all) {
        int x;
        if (n_frames >= 16) {
            x = xcd_of[items[u.t.item].frame];
        } else {
            x = least();
            load[x] += u.cost;
        }
        lists[x].push_back(u.t);
    }
    int n = 0;
    for (int x = 0; x < 8; ++x) {
        xs->start[x] = n;
        for (const Tile& t : lists[x]) out[n++] = t;
    }
    xs->start[8] = n;
    int g = ceil_div(std::max(n, 1), 8) * 8;
    const int cap = grid_cap > 0 ? std::max(8, grid_cap / 8 * 8) : S32_GRID_MAX;
    *grid = std::min(g, cap);
    return n;
}

// Table capacity for one level: the shortest bands over runs of 2 tiles, the
// finest the builder makes.
int64_t score32_band_capacity(int nx, int ny, int wc) {
    if (nx <= 0 || ny <= 0) return 0;
    return (int64_t)ceil_div(ny, 2 * s32_pairs(4)) * ceil_div(ceil_div(wc, S32_TILE), 2);
}

hipError_t launch_pack_score32(const float* w, int n_models, float* out, hipStream_t s) {
    const int n = n_models * S32_MODEL;
    pack32_kernel<<<ceil_div(n, 256), 256, 0, s>>>(w, n_models, out);
    return hipGetLastError();
}

hipError_t launch_score32_table(const LevelItem* items, const Tile* bands, const XcdLists& xs, int grid,
                                const float* packed, const float* bias, int n_models, int features, int rows,
                                int* ctr, const Decide32& dec, hipStream_t s) {
    if (xs.start[8] <= 0 || n_models <= 0) return hipSuccess;
    // the decisions need the max over the models, and the room of the shapes
    // of 8 and 16 row pairs per band
    if (dec.counters && (n_models != 1 || rows == 16)) return hipErrorInvalidValue;
    const dim3 g((unsigned)grid, (unsigned)n_models);
    switch (features & (PD_FEAT_HOG | PD_FEAT_LBP)) {
        case PD_FEAT_HOG: launch_feat<PD_FEAT_HOG>(rows, g, items, bands, xs, packed, bias, ctr, dec, s); break;
        case PD_FEAT_LBP: launch_feat<PD_FEAT_LBP>(rows, g, items, bands, xs, packed, bias, ctr, dec, s); break;
        default: launch_feat<PD_FEAT_HOG | PD_FEAT_LBP>(rows, g, items, bands, xs, packed, bias, ctr, dec, s); break;
    }
    return hipGetLastError();
}

}  // namespace pd
