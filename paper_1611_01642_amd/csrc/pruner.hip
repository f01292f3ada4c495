// The learned window pruner: a 68-32-32-16 conv3x3 network with a 1x1
// sigmoid head over the per-cell feature map of every pyramid level, trained
// on the GPU with these kernels.  The network is not part of the paper; it
// predicts which windows the linear SVM of Section 4.4 will score above the
// threshold, so the others need not be scored.
//
// Layout: every map is planar FP32 [C][hc][wc]; one item per map (a pyramid
// level of a frame) carries pointers to its cell map, activations, gradient
// buffers, logits, labels and mask.  Work tiles are 64 consecutive cells of
// one row; a wave owns a tile, a lane owns a cell.
//
//  * conv3x3 (zero padding): per input channel the wave stages the 3 x 66
//    neighbourhood of its tile in LDS (the next channel's loads in flight),
//    then each lane accumulates all output channels in registers with
//    wave-uniform weights (scalar loads, tap-major layout [cin][9][cout]).
//    The same kernel computes the data gradient with the flipped, transposed
//    weights and the ReLU mask of the layer below.  The last layer fuses the
//    1x1 head.
//  * weight gradients: dW[o][c][u][v] = sum over cells of dZ[o] x X[c] at
//    offset (u - 1, v - 1): a fixed set of workgroups strides over the tiles
//    (both operands staged in LDS), each thread owning one output channel and
//    a group of input channels; per-workgroup partials are then summed in
//    FP64 in a fixed order, so gradients are bitwise reproducible.
//  * loss: class-weighted binary cross-entropy over the masked cells; the
//    gradients are accumulated un-normalised and divided by the number of
//    masked cells in the final reduction.
#include <cmath>

#include <algorithm>

#include "pd_internal.h"

namespace pd {
namespace {

constexpr int NW = 64;  // cells per tile
constexpr int NWAVES = 4;
constexpr int HALO_W = NW + 2;

template <int COUT, bool HEAD>
__global__ void __launch_bounds__(256) conv3x3_kernel(const NetItem* __restrict__ items,
                                                      const Tile* __restrict__ tiles, int n_tiles, int in_slot,
                                                      int cin, int out_slot, int mask_slot,
                                                      const float* __restrict__ wt, const float* __restrict__ bias,
                                                      int relu, const float* __restrict__ head) {
    __shared__ float stage[NWAVES][2][3 * HALO_W];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int task = blockIdx.x * NWAVES + wave;
    if (task >= n_tiles) return;
    const Tile tl = tiles[task];
    const NetItem& it = items[tl.item];
    const int wc = it.wc, hc = it.hc;
    const int p = tl.ty, q0 = tl.tx * NW, q = q0 + lane;
    const size_t plane = (size_t)hc * wc;
    const float* in = it.buf[in_slot];

    float acc[COUT];
#pragma unroll
    for (int o = 0; o < COUT; ++o) acc[o] = bias ? bias[o] : 0.0f;

    // staged element e = r * 66 + col holds in[c][p - 1 + r][q0 - 1 + col] (0 outside)
    int off[4];
    bool ok[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = lane + 64 * k;
        const int r = e / HALO_W, col = e - (e / HALO_W) * HALO_W;
        const int y = p - 1 + r, x = q0 - 1 + col;
        ok[k] = e < 3 * HALO_W && y >= 0 && y < hc && x >= 0 && x < wc;
        off[k] = ok[k] ? y * wc + x : 0;
    }
    float pre[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) pre[k] = ok[k] ? in[off[k]] : 0.0f;
    for (int c = 0; c < cin; ++c) {
        float* s = stage[wave][c & 1];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (lane + 64 * k < 3 * HALO_W) s[lane + 64 * k] = pre[k];
        if (c + 1 < cin) {
            const float* nx = in + (size_t)(c + 1) * plane;
#pragma unroll
            for (int k = 0; k < 4; ++k) pre[k] = ok[k] ? nx[off[k]] : 0.0f;
        }
        __builtin_amdgcn_wave_barrier();
        float xv[9];
#pragma unroll
        for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int v = 0; v < 3; ++v) xv[u * 3 + v] = s[u * HALO_W + lane + v];
        const float* w = wt + (size_t)c * 9 * COUT;
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int o = 0; o < COUT; ++o) acc[o] = fmaf(xv[t], w[t * COUT + o], acc[o]);
        __builtin_amdgcn_wave_barrier();
    }
    if (q >= wc) return;
    const size_t at = (size_t)p * wc + q;
    if (relu) {
#pragma unroll
        for (int o = 0; o < COUT; ++o) acc[o] = fmaxf(acc[o], 0.0f);
    }
    if (mask_slot >= 0) {  // data gradient through the ReLU of the layer below
        const float* a = it.buf[mask_slot];
#pragma unroll
        for (int o = 0; o < COUT; ++o) acc[o] = a[o * plane + at] > 0.0f ? acc[o] : 0.0f;
    }
    if (out_slot >= 0) {
        float* out = it.buf[out_slot];
#pragma unroll
        for (int o = 0; o < COUT; ++o) out[o * plane + at] = acc[o];
    }
    if (HEAD) {
        float z = head[COUT];
#pragma unroll
        for (int o = 0; o < COUT; ++o) z = fmaf(head[o], acc[o], z);
        it.logit[at] = z;
    }
}

// dW partials of one layer: thread = (output channel o, channel group g).
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) wgrad_kernel(const NetItem* __restrict__ items, const Tile* __restrict__ tiles,
                                                    int n_tiles, int x_slot, int dz_slot,
                                                    float* __restrict__ partial) {
    constexpr int G = 256 / COUT;
    constexpr int CPT = (CIN + G - 1) / G;
    constexpr int NOUT = COUT * CIN * 9 + COUT;
    __shared__ float xs[CIN][3][HALO_W];
    __shared__ float ds[COUT][NW + 1];
    const int tid = threadIdx.x;
    const int o = tid % COUT, g = tid / COUT;
    float acc[CPT][9];
#pragma unroll
    for (int j = 0; j < CPT; ++j)
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[j][t] = 0.0f;
    float accb = 0.0f;
    for (int ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
        const Tile tl = tiles[ti];
        const NetItem& it = items[tl.item];
        const int wc = it.wc, hc = it.hc, p = tl.ty, q0 = tl.tx * NW;
        const size_t plane = (size_t)hc * wc;
        const float* x = it.buf[x_slot];
        const float* dz = it.buf[dz_slot];
        __syncthreads();  // the previous tile's reads are done
        for (int e = tid; e < CIN * 3 * HALO_W; e += 256) {
            const int c = e / (3 * HALO_W), rem = e - c * (3 * HALO_W);
            const int r = rem / HALO_W, col = rem - r * HALO_W;
            const int y = p - 1 + r, xx = q0 - 1 + col;
            xs[c][r][col] = (y >= 0 && y < hc && xx >= 0 && xx < wc) ? x[c * plane + (size_t)y * wc + xx] : 0.0f;
        }
        for (int e = tid; e < COUT * NW; e += 256) {
            const int oo = e / NW, qq = e - oo * NW;
            ds[oo][qq] = q0 + qq < wc ? dz[oo * plane + (size_t)p * wc + q0 + qq] : 0.0f;
        }
        __syncthreads();
        for (int qq = 0; qq < NW; ++qq) {
            const float d = ds[o][qq];
            accb += d;
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const int c = g + G * j;
                if (c < CIN) {
#pragma unroll
                    for (int u = 0; u < 3; ++u)
#pragma unroll
                        for (int v = 0; v < 3; ++v) acc[j][u * 3 + v] = fmaf(d, xs[c][u][qq + v], acc[j][u * 3 + v]);
                }
            }
        }
    }
    float* out = partial + (size_t)blockIdx.x * NOUT;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int c = g + G * j;
        if (c < CIN) {
#pragma unroll
            for (int t = 0; t < 9; ++t) out[(o * CIN + c) * 9 + t] = acc[j][t];
        }
    }
    if (g == 0) out[COUT * CIN * 9 + o] = accb;
}

// Loss and head: per cell dz = m((1 - y) s - pw y (1 - s)) (un-normalised),
// dZ3[c] = dz hw[c] [a3[c] > 0]; per-workgroup partials of dhw, dhb, the
// loss and the number of masked cells (NHEAD = 16 + 3 values).
constexpr int HEAD_C = 16;
constexpr int NHEAD = HEAD_C + 3;

__device__ __forceinline__ float softplus(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }

__global__ void __launch_bounds__(256) head_loss_kernel(const NetItem* __restrict__ items,
                                                        const Tile* __restrict__ tiles, int n_tiles, int a3_slot,
                                                        int dz_slot, const float* __restrict__ head, float pos_weight,
                                                        double* __restrict__ partial) {
    __shared__ double red[256][NHEAD];
    double mine[NHEAD];
#pragma unroll
    for (int k = 0; k < NHEAD; ++k) mine[k] = 0.0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int task = blockIdx.x * NWAVES + wave;
    if (task < n_tiles) {
        const Tile tl = tiles[task];
        const NetItem& it = items[tl.item];
        const int q = tl.tx * NW + lane;
        if (q < it.wc) {
            const size_t plane = (size_t)it.hc * it.wc;
            const size_t at = (size_t)tl.ty * it.wc + q;
            const float z = it.logit[at], y = it.label[at], m = it.mask[at];
            const float s = 1.0f / (1.0f + expf(-z));
            const float dz = m * ((1.0f - y) * s - pos_weight * y * (1.0f - s));
            const float* a3 = it.buf[a3_slot];
            float* dz3 = it.buf[dz_slot];
#pragma unroll
            for (int c = 0; c < HEAD_C; ++c) {
                const float a = a3[c * plane + at];
                dz3[c * plane + at] = a > 0.0f ? dz * head[c] : 0.0f;
                mine[c] = (double)dz * (double)a;
            }
            mine[HEAD_C] = dz;
            mine[HEAD_C + 1] = m != 0.0f ? (double)m * ((double)pos_weight * y * softplus(-z) +
                                                         (1.0 - (double)y) * softplus(z))
                                         : 0.0;
            mine[HEAD_C + 2] = m;
        }
    }
#pragma unroll
    for (int k = 0; k < NHEAD; ++k) red[threadIdx.x][k] = mine[k];
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride)
            for (int k = 0; k < NHEAD; ++k) red[threadIdx.x][k] += red[threadIdx.x + stride][k];
        __syncthreads();
    }
    if (threadIdx.x < NHEAD) partial[(size_t)blockIdx.x * NHEAD + threadIdx.x] = red[0][threadIdx.x];
}

// Head partials -> grad of hw and hb (divided by N), loss, N.
__global__ void head_reduce_kernel(const double* __restrict__ partial, int n_blocks, float* __restrict__ grad_head,
                                   double* __restrict__ stats) {
    const int k = threadIdx.x;
    if (k >= NHEAD) return;
    double s = 0.0;
    for (int b = 0; b < n_blocks; ++b) s += partial[(size_t)b * NHEAD + k];
    __shared__ double sums[NHEAD];
    sums[k] = s;
    __syncthreads();
    const double n = sums[HEAD_C + 2];
    const double inv = n > 0.0 ? 1.0 / n : 0.0;
    if (k <= HEAD_C) grad_head[k] = (float)(s * inv);
    if (k == HEAD_C + 1) stats[0] = s * inv;  // mean loss
    if (k == HEAD_C + 2) stats[1] = n;        // masked cells
}

// Layer partials -> gradient slice (divided by N = stats[1]).
__global__ void __launch_bounds__(256) wgrad_reduce_kernel(const float* __restrict__ partial, int n_blocks, int nout,
                                                           const double* __restrict__ stats,
                                                           float* __restrict__ grad) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= nout) return;
    double s = 0.0;
    for (int b = 0; b < n_blocks; ++b) s += (double)partial[(size_t)b * nout + k];
    const double n = stats[1];
    grad[k] = (float)(n > 0.0 ? s / n : 0.0);
}

// Tap-major copies of the conv weights: forward [cin][9][cout], and the
// flipped, transposed form [cout][9][cin] used for data gradients.
__global__ void __launch_bounds__(256) prep_weights_kernel(const float* __restrict__ params, float* __restrict__ fwd,
                                                           float* __restrict__ bwd, int cin, int cout) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= cout * cin * 9) return;
    const int o = e / (cin * 9), rem = e - o * cin * 9, c = rem / 9, t = rem - c * 9;
    const float w = params[e];
    fwd[((size_t)c * 9 + t) * cout + o] = w;
    if (bwd) bwd[((size_t)o * 9 + (8 - t)) * cin + c] = w;
}

__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + eps);
}

__global__ void __launch_bounds__(256) window_labels_kernel(const float* __restrict__ scores, int nx, int ny,
                                                            int wc, int hc, const double* __restrict__ thr,
                                                            float* __restrict__ labels, float* __restrict__ mask) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= wc * hc) return;
    const int cy = e / wc, cx = e - cy * wc;
    const int i = cy - PRUNER_WIN_DI, j = cx - PRUNER_WIN_DJ;
    const bool win = i >= 0 && i < ny && j >= 0 && j < nx;
    mask[e] = win ? 1.0f : 0.0f;
    labels[e] = win && (double)scores[(size_t)i * nx + j] > thr[0] ? 1.0f : 0.0f;
}

// ---- BF16 MFMA inference ------------------------------------------------------
// Implicit GEMM per layer on v_mfma_f32_16x16x32_bf16: M = 16 cells of a row,
// N = 16 output channels, K = (tap, input channel) with the channel vector of
// each neighbour cell contiguous (channels-last maps).  Persistent workgroups:
// each wave loads the packed weight fragments of its output-channel tile into
// registers once, then the workgroup loops over tiles of 2 rows x 64 cells,
// staging the 4 x 66 input cells in LDS per tile (a contiguous run of the
// table per workgroup); the waves sharing an
// output-channel tile split its 8 M-tiles.  FP32 accumulation over K in
// ascending order; bias and ReLU in FP32, outputs rounded to BF16; the last
// layer applies the 1x1 head (cross-lane sum over its 16 channels) and writes
// FP32 logits.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int L>
struct Layer;
template <>
struct Layer<1> {
    static constexpr int CIN = 68, CP = PR_CP1, XS = PR_CP1, COUT = 32;
};
template <>
struct Layer<2> {
    static constexpr int CIN = 32, CP = 32, XS = 40, COUT = 32;
};
template <>
struct Layer<3> {
    static constexpr int CIN = 32, CP = 32, XS = 40, COUT = 16;
};
template <int L>
struct LayerDims : Layer<L> {
    static constexpr int KCH = (9 * Layer<L>::CP + 31) / 32;  // K chunks of 32
    static constexpr int NT = Layer<L>::COUT / 16;            // N tiles
    static constexpr int PACKED = KCH * NT * 64 * 8;          // bf16 values
    static constexpr int PARAMS = Layer<L>::COUT * Layer<L>::CIN * 9;
};

constexpr int MR = 2;           // output rows per workgroup
constexpr int MC = 64;          // output cells per row
constexpr int XR = MR + 2, XC = MC + 2;

template <int L>
__global__ void __launch_bounds__(256) pack_bf16_kernel(const float* __restrict__ w, uint16_t* __restrict__ out) {
    using D = LayerDims<L>;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= D::PACKED) return;
    const int t = e / (D::NT * 512), n = (e / 512) % D::NT, l = (e / 8) % 64, j = e % 8;
    const int k = 32 * t + 8 * (l >> 4) + j, och = 16 * n + (l & 15);
    const int tap = k / D::CP, c = k - tap * D::CP;
    const float v = (tap < 9 && c < D::CIN) ? w[((size_t)och * D::CIN + c) * 9 + tap] : 0.0f;
    out[e] = f32_to_bf16(v);
}

template <int L>
__global__ void __launch_bounds__(256) conv_mfma_kernel(const LevelItem* __restrict__ items,
                                                        const Tile* __restrict__ tiles, int n_tiles,
                                                        const uint16_t* __restrict__ packed,
                                                        const float* __restrict__ bias,
                                                        const float* __restrict__ head) {
    using D = LayerDims<L>;
    constexpr int CP = D::CP, XS = D::XS, KCH = D::KCH, NT = D::NT;
    constexpr int WPN = 4 / NT;                  // waves per output-channel tile
    constexpr int MT = (MR * MC / 16) / WPN;     // M-tiles per wave
    static_assert(MT * WPN * 16 == MR * MC && (MC / 16) % MT == 0, "a wave's M-tiles lie in one row");
    __shared__ __attribute__((aligned(16))) uint16_t xs[XR * XC * XS];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int nw = wave % NT;                    // this wave's output-channel tile
    const int m0 = (wave / NT) * MT;             // its first M-tile (row-major over MR x MC / 16)
    const int prow = m0 / (MC / 16), cbase = (m0 % (MC / 16)) * 16;

    // this wave's B fragments, fragment order (K chunk t, N tile nw, lane)
    u32x4 bw[KCH];
#pragma unroll
    for (int t = 0; t < KCH; ++t) bw[t] = reinterpret_cast<const u32x4*>(packed)[(t * NT + nw) * 64 + lane];

    // a contiguous run of the (row-major) tile table per workgroup, so the
    // input rows a tile shares with the previous row pair are still in this
    // XCD's L2
    const int run = (n_tiles + gridDim.x - 1) / gridDim.x;
    const int t_end = min(n_tiles, ((int)blockIdx.x + 1) * run);
    // the (MR + 2) x (MC + 2) input cells of a tile, zero outside the map, into
    // registers; the next tile's loads are issued before this tile's MFMAs
    // (software pipeline: the loads are in flight while the matrix cores run)
    constexpr int PARTS = CP / 8;
    constexpr int NXQ = (XR * XC * PARTS + 255) / 256;
    u32x4 xv[NXQ];
    auto load_tile = [&](int ti) __attribute__((always_inline)) {
        const Tile tl = tiles[ti];
        const LevelItem& it = items[tl.item];
        const int wc = it.wc, hc = it.hc;
        const int p0 = tl.ty * MR, q0 = tl.tx * MC;
        const uint16_t* in = L == 1 ? it.cmap16 : (L == 2 ? it.act1 : it.act2);
#pragma unroll
        for (int k = 0; k < NXQ; ++k) {
            const int e = tid + 256 * k;
            const int cell = e / PARTS, part = e - cell * PARTS;
            const int r = cell / XC, col = cell - r * XC;
            const int y = p0 - 1 + r, x = q0 - 1 + col;
            xv[k] = u32x4{0u, 0u, 0u, 0u};
            if (e < XR * XC * PARTS && y >= 0 && y < hc && x >= 0 && x < wc)
                xv[k] = *reinterpret_cast<const u32x4*>(in + ((size_t)y * wc + x) * CP + 8 * part);
        }
    };
    if ((int)blockIdx.x * run < t_end) load_tile(blockIdx.x * run);
    for (int ti = blockIdx.x * run; ti < t_end; ++ti) {
        const Tile tl = tiles[ti];
        const LevelItem& it = items[tl.item];
        const int wc = it.wc, hc = it.hc;
        const int p0 = tl.ty * MR, q0 = tl.tx * MC;
        __syncthreads();  // the previous tile's reads of xs are done
#pragma unroll
        for (int k = 0; k < NXQ; ++k) {
            const int e = tid + 256 * k;
            if (e < XR * XC * PARTS) {
                const int cell = e / PARTS, part = e - cell * PARTS;
                *reinterpret_cast<u32x4*>(xs + cell * XS + 8 * part) = xv[k];
            }
        }
        __syncthreads();
        if (ti + 1 < t_end) load_tile(ti + 1);

        f32x4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < KCH; ++t) {
            const int k0 = 32 * t + 8 * (lane >> 4);
            const int tap = k0 / CP, c0 = k0 - tap * CP;
            const int u = tap / 3, v = tap - 3 * (tap / 3);
            const bf16x8 b = __builtin_bit_cast(bf16x8, bw[t]);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int col = cbase + 16 * mt + (lane & 15);
                u32x4 av = {0u, 0u, 0u, 0u};
                if (tap < 9) av = *reinterpret_cast<const u32x4*>(xs + ((prow + u) * XC + col + v) * XS + c0);
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), b, acc[mt], 0, 0, 0);
            }
        }

        // lane holds D[cell 4 * (lane / 16) + r][channel lane % 16] of each tile
        const int p = p0 + prow;
        const int och = 16 * nw + (lane & 15);
        if (L < 3) {
            uint16_t* out = L == 1 ? it.act1 : it.act2;
            const float bo = bias[och];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int q = q0 + cbase + 16 * mt + 4 * (lane >> 4) + r;
                    if (p < hc && q < wc) out[((size_t)p * wc + q) * 32 + och] = f32_to_bf16(fmaxf(acc[mt][r] + bo, 0.0f));
                }
        } else {
            const float bo = bias[och], hw = head[och], hb = head[16];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float z = hw * fmaxf(acc[mt][r] + bo, 0.0f);
                    z += __shfl_xor(z, 8, 16);
                    z += __shfl_xor(z, 4, 16);
                    z += __shfl_xor(z, 2, 16);
                    z += __shfl_xor(z, 1, 16);
                    const int q = q0 + cbase + 16 * mt + 4 * (lane >> 4) + r;
                    if ((lane & 15) == 0 && p < hc && q < wc) it.logit[(size_t)p * wc + q] = z + hb;
                }
        }
    }
}

}  // namespace

int64_t pruner_prep_floats() {
    int64_t n = 0;
    for (int l = 0; l < 3; ++l) n += 2LL * PRUNER_CH[l] * PRUNER_CH[l + 1] * 9;
    return n;
}

hipError_t launch_pruner_prep(const float* params, float* prep, hipStream_t s) {
    const float* src = params;
    float* dst = prep;
    for (int l = 0; l < 3; ++l) {
        const int cin = PRUNER_CH[l], cout = PRUNER_CH[l + 1], n = cin * cout * 9;
        prep_weights_kernel<<<ceil_div(n, 256), 256, 0, s>>>(src, dst, dst + n, cin, cout);
        src += n + cout;
        dst += 2 * n;
    }
    return hipGetLastError();
}

hipError_t launch_pruner_forward(const NetItem* items, const Tile* tiles, int n_tiles, const float* params,
                                 const float* prep, bool keep_a3, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    const int grid = ceil_div(n_tiles, NWAVES);
    const float* b1 = params + 68 * 32 * 9;
    const float* b2 = b1 + 32 + 32 * 32 * 9;
    const float* b3 = b2 + 32 + 32 * 16 * 9;
    const float* head = b3 + 16;
    const float* w1 = prep;
    const float* w2 = w1 + 2 * 68 * 32 * 9;
    const float* w3 = w2 + 2 * 32 * 32 * 9;
    conv3x3_kernel<32, false><<<grid, 256, 0, s>>>(items, tiles, n_tiles, NET_X, 68, NET_A1, -1, w1, b1, 1, nullptr);
    conv3x3_kernel<32, false><<<grid, 256, 0, s>>>(items, tiles, n_tiles, NET_A1, 32, NET_A2, -1, w2, b2, 1, nullptr);
    conv3x3_kernel<16, true><<<grid, 256, 0, s>>>(items, tiles, n_tiles, NET_A2, 32, keep_a3 ? NET_A3 : -1, -1, w3,
                                                  b3, 1, head);
    return hipGetLastError();
}

int pruner_wgrad_blocks(int n_tiles) { return n_tiles < 1 ? 1 : (n_tiles < 512 ? n_tiles : 512); }

int64_t pruner_partial_floats(int n_tiles) {
    // the largest layer's partials, reused by each layer in turn (+ head, as doubles)
    const int nb = pruner_wgrad_blocks(n_tiles);
    return (int64_t)nb * (68 * 32 * 9 + 32) + 2LL * ceil_div(n_tiles, NWAVES) * NHEAD + 4;
}

hipError_t launch_pruner_backward(const NetItem* items, const Tile* tiles, int n_tiles, const float* params,
                                  const float* prep, float pos_weight, float* grad, double* stats, float* partial,
                                  hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    const int grid = ceil_div(n_tiles, NWAVES);
    const int nb = pruner_wgrad_blocks(n_tiles);
    const int n1 = 68 * 32 * 9, n2 = 32 * 32 * 9, n3 = 32 * 16 * 9;
    const float* head = params + n1 + 32 + n2 + 32 + n3 + 16;
    const float* w2b = prep + 2 * n1 + n2;
    const float* w3b = prep + 2 * n1 + 2 * n2 + n3;
    float* g1 = grad;
    float* g2 = g1 + n1 + 32;
    float* g3 = g2 + n2 + 32;
    float* gh = g3 + n3 + 16;
    double* hpart = reinterpret_cast<double*>(partial + (int64_t)nb * (n1 + 32));
    // head and loss, then the normaliser N
    head_loss_kernel<<<grid, 256, 0, s>>>(items, tiles, n_tiles, NET_A3, NET_GA, head, pos_weight, hpart);
    head_reduce_kernel<<<1, 64, 0, s>>>(hpart, grid, gh, stats);
    // layer 3: dW3 from dZ3 (GA) and a2; dZ2 = conv(dZ3, W3 flipped) [a2 > 0] -> GB
    wgrad_kernel<32, 16><<<nb, 256, 0, s>>>(items, tiles, n_tiles, NET_A2, NET_GA, partial);
    wgrad_reduce_kernel<<<ceil_div(n3 + 16, 256), 256, 0, s>>>(partial, nb, n3 + 16, stats, g3);
    conv3x3_kernel<32, false><<<grid, 256, 0, s>>>(items, tiles, n_tiles, NET_GA, 16, NET_GB, NET_A2, w3b, nullptr, 0,
                                                   nullptr);
    // layer 2: dW2 from dZ2 (GB) and a1; dZ1 = conv(dZ2, W2 flipped) [a1 > 0] -> GA
    wgrad_kernel<32, 32><<<nb, 256, 0, s>>>(items, tiles, n_tiles, NET_A1, NET_GB, partial);
    wgrad_reduce_kernel<<<ceil_div(n2 + 32, 256), 256, 0, s>>>(partial, nb, n2 + 32, stats, g2);
    conv3x3_kernel<32, false><<<grid, 256, 0, s>>>(items, tiles, n_tiles, NET_GB, 32, NET_GA, NET_A1, w2b, nullptr, 0,
                                                   nullptr);
    // layer 1: dW1 from dZ1 (GA) and the cell map
    wgrad_kernel<68, 32><<<nb, 256, 0, s>>>(items, tiles, n_tiles, NET_X, NET_GA, partial);
    wgrad_reduce_kernel<<<ceil_div(n1 + 32, 256), 256, 0, s>>>(partial, nb, n1 + 32, stats, g1);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, int step, float lr, float b1, float b2,
                       float eps, hipStream_t s) {
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, step)));
    adam_kernel<<<ceil_div(n, 256), 256, 0, s>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_window_labels(const float* scores, int nx, int ny, int wc, int hc, const double* thr,
                                float* labels, float* mask, hipStream_t s) {
    window_labels_kernel<<<ceil_div(wc * hc, 256), 256, 0, s>>>(scores, nx, ny, wc, hc, thr, labels, mask);
    return hipGetLastError();
}

int64_t pruner_packed_bf16_elems() {
    return (int64_t)LayerDims<1>::PACKED + LayerDims<2>::PACKED + LayerDims<3>::PACKED;
}

hipError_t launch_pruner_pack_bf16(const float* params, uint16_t* packed, hipStream_t s) {
    const float* w1 = params;
    const float* w2 = w1 + LayerDims<1>::PARAMS + 32;
    const float* w3 = w2 + LayerDims<2>::PARAMS + 32;
    pack_bf16_kernel<1><<<ceil_div(LayerDims<1>::PACKED, 256), 256, 0, s>>>(w1, packed);
    pack_bf16_kernel<2><<<ceil_div(LayerDims<2>::PACKED, 256), 256, 0, s>>>(w2, packed + LayerDims<1>::PACKED);
    pack_bf16_kernel<3><<<ceil_div(LayerDims<3>::PACKED, 256), 256, 0, s>>>(
        w3, packed + LayerDims<1>::PACKED + LayerDims<2>::PACKED);
    return hipGetLastError();
}

int pruner_mfma_tiles_y(int hc) { return ceil_div(hc, MR); }

hipError_t launch_pruner_mfma(const LevelItem* items, const Tile* tiles, int n_tiles, const float* params,
                              const uint16_t* packed, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    const float* b1 = params + LayerDims<1>::PARAMS;
    const float* b2 = b1 + 32 + LayerDims<2>::PARAMS;
    const float* b3 = b2 + 32 + LayerDims<3>::PARAMS;
    const float* head = b3 + 16;
    // persistent workgroups: a few per CU, each looping over the tiles
    const int grid = std::min(n_tiles, 4 * 256);
    conv_mfma_kernel<1><<<grid, 256, 0, s>>>(items, tiles, n_tiles, packed, b1, nullptr);
    conv_mfma_kernel<2><<<grid, 256, 0, s>>>(items, tiles, n_tiles, packed + LayerDims<1>::PACKED, b2, nullptr);
    conv_mfma_kernel<3><<<grid, 256, 0, s>>>(items, tiles, n_tiles,
                                             packed + LayerDims<1>::PACKED + LayerDims<2>::PACKED, b3, head);
    return hipGetLastError();
}

namespace {

// Order-preserving map of a float to an unsigned key (larger float, larger key).
__device__ __forceinline__ uint32_t fkey(float z) {
    const uint32_t u = __float_as_uint(z + 0.0f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// One workgroup per frame: radix selection (8 bits per pass, most significant
// first) of the K-th largest logit over the frame's windows, every level.
constexpr int TOPK_BATCH = 8;

__global__ void __launch_bounds__(256) topk_kernel(const LevelItem* __restrict__ items,
                                                   const int32_t* __restrict__ first_item,
                                                   const NmsGeom* __restrict__ geoms, int keep_k,
                                                   float* __restrict__ kth) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t sel[2];  // prefix, remaining rank
    __shared__ int total_s;
    const int f = blockIdx.x, tid = threadIdx.x;
    const int i0 = first_item[f], nl = geoms[f].n_levels;
    if (tid == 0) {
        int n = 0;
        for (int l = 0; l < nl; ++l) n += items[i0 + l].nx * items[i0 + l].ny;
        total_s = n;
        sel[0] = 0u;
        sel[1] = (uint32_t)keep_k;
    }
    __syncthreads();
    if (keep_k >= total_s) {  // every window is kept
        if (tid == 0) kth[f] = -INFINITY;
        return;
    }
    uint32_t mask = 0u;
    for (int shift = 24; shift >= 0; shift -= 8) {
        hist[tid] = 0u;
        __syncthreads();
        const uint32_t prefix = sel[0];
        for (int l = 0; l < nl; ++l) {
            const LevelItem& it = items[i0 + l];
            const int n = it.nx * it.ny;
            // eight logit loads of a thread in flight together
            for (int q0 = tid; q0 < n; q0 += 256 * TOPK_BATCH) {
                uint32_t k[TOPK_BATCH];
#pragma unroll
                for (int u = 0; u < TOPK_BATCH; ++u) {
                    const int q = min(q0 + 256 * u, n - 1);
                    const int wi = q / it.nx, wj = q - wi * it.nx;
                    k[u] = fkey(it.logit[(size_t)(wi + PRUNER_WIN_DI) * it.wc + wj + PRUNER_WIN_DJ]);
                }
#pragma unroll
                for (int u = 0; u < TOPK_BATCH; ++u)
                    if (q0 + 256 * u < n && (k[u] & mask) == prefix) atomicAdd(&hist[(k[u] >> shift) & 255u], 1u);
            }
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t rank = sel[1], d = 255u;
            for (;; --d) {
                if (hist[d] >= rank || d == 0u) break;
                rank -= hist[d];
            }
            sel[0] = prefix | (d << shift);
            sel[1] = rank;
        }
        mask |= 255u << shift;
        __syncthreads();
    }
    if (tid == 0) {
        const uint32_t k = sel[0];
        kth[f] = __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
    }
}

// One wave per score tile: does any of its windows have logit >= kth?
__global__ void __launch_bounds__(256) tile_filter_kernel(const LevelItem* __restrict__ items,
                                                          const Tile* __restrict__ tiles, int n_tiles, int rows,
                                                          int cols, const float* __restrict__ kth,
                                                          Tile* __restrict__ kept, int32_t* __restrict__ kept_count) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t = blockIdx.x * 4 + wave;
    if (t >= n_tiles) return;
    const Tile tl = tiles[t];
    const LevelItem& it = items[tl.item];
    const float thr = kth[it.frame];
    // a tile of width w < cols (FP32 lane groups) covers cols / w row chunks
    const int w = cols == SC_W ? tile_width(tl) : cols;
    const int r0 = tl.ty * rows, nr = rows * (cols / w);
    bool any = false;
    for (int c = lane; c < w; c += 64) {
        const int j = tl.tx * cols + c;
        if (j >= it.nx) break;
        for (int r = 0; r < nr; ++r) {
            const int i = r0 + r;
            if (i >= it.ny) break;
            any = any || it.logit[(size_t)(i + PRUNER_WIN_DI) * it.wc + j + PRUNER_WIN_DJ] >= thr;
        }
    }
    if (__any(any) && lane == 0) kept[atomicAdd(kept_count, 1)] = tl;
}

}  // namespace

hipError_t launch_topk(const LevelItem* items, const int32_t* first_item, const NmsGeom* geoms, int n_frames,
                       int keep_k, float* kth, hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    topk_kernel<<<n_frames, 256, 0, s>>>(items, first_item, geoms, keep_k, kth);
    return hipGetLastError();
}

hipError_t launch_tile_filter(const LevelItem* items, const Tile* tiles, int n_tiles, int rows, int cols,
                              const float* kth, Tile* kept, int32_t* kept_count, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    tile_filter_kernel<<<ceil_div(n_tiles, 4), 256, 0, s>>>(items, tiles, n_tiles, rows, cols, kth, kept, kept_count);
    return hipGetLastError();
}

}  // namespace pd
