// Threshold classification (Section 4.4) and non-maximum-suppression
// refinement (Section 3; Section 4.1 step 5, done here on the GPU).
//
// compact: four windows per thread, their loads in flight together; a
//   window's score is the max over the models (lowest model index on ties);
//   windows with score > threshold are appended to their frame's candidate
//   list with an atomic counter.  A frame's list has room for every one of
//   its windows, so none is dropped.
// select: for a frame with more than PD_MAX_CANDIDATES candidates, the
//   PD_MAX_CANDIDATES highest-scoring ones (score descending, then level, i,
//   j ascending: a strict order, keys are distinct) by a radix select over
//   the 64-bit NMS sort key; the selected set does not depend on the order
//   in which compaction appended the list.
// nms: one workgroup (16 waves) per frame.  Candidates are sorted by (score descending,
//   level, i, j ascending) with a bitonic sort in LDS; the greedy pass walks
//   them in chunks of 64: a candidate is suppressed if it overlaps (IoU > 0.5,
//   decided exactly as 2*inter > union on integer boxes) a box kept in an
//   earlier chunk (tested in parallel; per-candidate flags, no atomics) or an
//   earlier kept box of its own chunk (a 64x64 overlap mask, one row per lane,
//   walked in order on the scalar unit).  This is exactly the serial greedy
//   algorithm, and needs no n x n mask in memory.
#include "pd_internal.h"

namespace pd {
namespace {

__global__ void zero_kernel(int32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void __launch_bounds__(CP_THREADS) compact_kernel(const LevelItem* __restrict__ items,
                                                             const Tile* __restrict__ tiles, int n_models,
                                                             const double* __restrict__ thresholds, float margin,
                                                             int32_t* __restrict__ counters,
                                                             float* __restrict__ cand_score,
                                                             int4* __restrict__ cand_key, double* __restrict__ cand_s64,
                                                             int32_t* __restrict__ near_count,
                                                             int4* __restrict__ near_key, int64_t near_cap, int n_frames,
                                                             const float* __restrict__ kth) {
    const Tile tl = tiles[blockIdx.x];
    const LevelItem& it = items[tl.item];
    const int n = it.nx * it.ny;
    const int q0 = tl.tx * CP_N + threadIdx.x;
    if (q0 >= n) return;
    // windows q0 + k * CP_THREADS: every load is issued before the first
    // decision (windows past the level read its last one and are skipped)
    int qk[CP_PER];
    float best[CP_PER];
    int bm[CP_PER];
    bool keep[CP_PER];
#pragma unroll
    for (int k = 0; k < CP_PER; ++k) {
        qk[k] = min(q0 + k * CP_THREADS, n - 1);
        best[k] = it.scores[qk[k]];
        bm[k] = 0;
        keep[k] = true;
        if (kth) {  // pruned: only windows the network keeps can be detections
            const int wi = qk[k] / it.nx, wj = qk[k] - wi * it.nx;
            keep[k] = it.logit[(size_t)(wi + PRUNER_WIN_DI) * it.wc + wj + PRUNER_WIN_DJ] >= kth[it.frame];
        }
    }
    for (int m = 1; m < n_models; ++m) {
#pragma unroll
        for (int k = 0; k < CP_PER; ++k) {
            const float v = it.scores[(size_t)m * n + qk[k]];
            if (v > best[k]) {
                best[k] = v;
                bm[k] = m;
            }
        }
    }
    const double thr = thresholds[it.frame];
#pragma unroll
    for (int k = 0; k < CP_PER; ++k) {
        const int q = q0 + k * CP_THREADS;
        if (q >= n || !keep[k]) continue;
        const int i = q / it.nx;
        if (margin > 0.0f && fabs((double)best[k] - thr) < (double)margin) {
            // too close to call in this precision: rescored in FP64.  near_count
            // holds one counter per frame and, after them, the length of the
            // dense list of all frames' near windows (room for every window of
            // the batch: the bound is never reached)
            atomicAdd(&near_count[it.frame], 1);
            const int g = atomicAdd(&near_count[n_frames], 1);
            if (g < near_cap) near_key[g] = make_int4(it.frame * PD_MAX_LEVELS + it.level, i, q - i * it.nx, bm[k]);
        } else if ((double)best[k] > thr) {
            const int pos = atomicAdd(&counters[it.frame], 1);
            if (pos < it.cand_cap) {  // always: a window is appended once at most
                const size_t o = (size_t)it.cand_off + pos;
                cand_score[o] = best[k];
                cand_key[o] = make_int4(it.level, i, q - i * it.nx, bm[k]);
                if (cand_s64) cand_s64[o] = __longlong_as_double(0x7ff8000000000000LL);
            }
        }
    }
}

// One workgroup of 16 waves per frame: the frame's LDS scratch allows one
// workgroup per compute unit, and the overlap tests and the sort are
// latency-bound, so the workgroup brings its own waves to hide the latency.
constexpr int NMS_WAVES = 16;
constexpr int NMS_THREADS = NMS_WAVES * 64;

struct NmsSmem {
    unsigned long long key[PD_MAX_CANDIDATES];
    uint16_t sidx[PD_MAX_CANDIDATES];
    uint16_t kpos[PD_MAX_CANDIDATES];
    int4 kbox[PD_MAX_CANDIDATES];
    int4 cbox[64];
    unsigned long long cmask[64];  // in-chunk overlap bits: candidate q's later overlaps
    uint32_t supf[64];  // candidate of the chunk overlaps an earlier kept box (every writer stores 1)
    int nkept;
};

__device__ inline unsigned long long sort_key(float s, int4 k) {
    s = s + 0.0f;  // -0 -> +0
    uint32_t f = __float_as_uint(s);
    f = (f & 0x80000000u) ? ~f : (f | 0x80000000u);  // ascending with the float
    const uint32_t lo = ((uint32_t)k.x << 22) | ((uint32_t)k.y << 11) | (uint32_t)k.z;
    // descending score first; real keys stay below the all-ones padding key
    return ((unsigned long long)min(~f, 0xFFFFFFFEu) << 32) | lo;
}

__device__ inline int4 window_box(const NmsGeom& g, int level, int i, int j) {
    level = min(max(level, 0), g.n_levels - 1);
    const int64_t w0 = g.wh[0][0], h0 = g.wh[0][1];
    const int64_t wk = g.wh[level][0], hk = g.wh[level][1];
    int4 b;
    b.x = (int)((256LL * PD_CELL * j * w0) / wk);
    b.y = (int)((256LL * PD_CELL * i * h0) / hk);
    b.z = (int)((256LL * (PD_CELL * j + PD_WIN_W) * w0) / wk);
    b.w = (int)((256LL * (PD_CELL * i + PD_WIN_H) * h0) / hk);
    return b;
}

// 2 * inter > union on the integer Q8 boxes.  Sides are below 2^23, so
// every product and sum here is an integer below 2^53: exact in FP64.
__device__ inline bool overlaps(const int4& a, const int4& b) {
    const int iw = min(a.z, b.z) - max(a.x, b.x);
    const int ih = min(a.w, b.w) - max(a.y, b.y);
    if (iw <= 0 || ih <= 0) return false;
    const double inter = (double)iw * (double)ih;
    const double uni = (double)(a.z - a.x) * (double)(a.w - a.y) + (double)(b.z - b.x) * (double)(b.w - b.y) - inter;
    return 2.0 * inter > uni;
}

// One workgroup per frame.  Finds the PD_MAX_CANDIDATES-th smallest key of
// the frame's list, one byte per pass from the top (LDS histogram of the
// keys that share the bytes found so far), then copies every entry whose key
// is at most that one: exactly PD_MAX_CANDIDATES entries, the keys being
// distinct.  Their order in the output is immaterial (NMS sorts by key).
constexpr int SEL_THREADS = 1024;

__global__ void __launch_bounds__(SEL_THREADS) cand_select_kernel(const NmsGeom* __restrict__ geoms,
                                                                  const int32_t* __restrict__ counters,
                                                                  const float* __restrict__ cand_score,
                                                                  const int4* __restrict__ cand_key,
                                                                  const double* __restrict__ cand_s64,
                                                                  float* __restrict__ sel_score,
                                                                  int4* __restrict__ sel_key,
                                                                  double* __restrict__ sel_s64) {
    const int f = blockIdx.x, t = threadIdx.x;
    const int n = min(counters[f], geoms[f].cand_cap);
    if (n <= PD_MAX_CANDIDATES) return;
    const size_t base = (size_t)geoms[f].cand_off;
    const float* cs = cand_score + base;
    const int4* ck = cand_key + base;
    __shared__ uint32_t hist[256];
    __shared__ unsigned long long s_prefix;
    __shared__ int s_rank, s_out;
    unsigned long long prefix = 0ull, mask = 0ull;
    int rank = PD_MAX_CANDIDATES;  // 1-based rank sought among the keys matching prefix
    for (int shift = 56; shift >= 0; shift -= 8) {
        if (t < 256) hist[t] = 0u;
        __syncthreads();
        for (int q = t; q < n; q += SEL_THREADS) {
            const unsigned long long key = sort_key(cs[q], ck[q]);
            if ((key & mask) == prefix) atomicAdd(&hist[(uint32_t)(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (t == 0) {
            int acc = 0, d = 0;
            for (; d < 255; ++d) {
                if (acc + (int)hist[d] >= rank) break;
                acc += (int)hist[d];
            }
            s_rank = rank - acc;
            s_prefix = prefix | ((unsigned long long)d << shift);
        }
        __syncthreads();
        rank = s_rank;
        prefix = s_prefix;
        mask |= 255ull << shift;
        __syncthreads();  // s_rank / s_prefix are rewritten by the next pass
    }
    if (t == 0) s_out = 0;
    __syncthreads();
    const size_t o = (size_t)f * PD_MAX_CANDIDATES;
    for (int q = t; q < n; q += SEL_THREADS) {
        if (sort_key(cs[q], ck[q]) <= prefix) {
            const int pos = atomicAdd(&s_out, 1);
            if (pos < PD_MAX_CANDIDATES) {
                sel_score[o + pos] = cs[q];
                sel_key[o + pos] = ck[q];
                if (sel_s64) sel_s64[o + pos] = cand_s64[base + q];
            }
        }
    }
}

__device__ void nms_frame(const NmsGeom& g, int frame, int raw_count, const float* __restrict__ cs,
                          const int4* __restrict__ ck, const double* __restrict__ c64, int rescored,
                          pd_box* __restrict__ boxes, int cap, pd_counts* __restrict__ counts) {
    extern __shared__ __align__(16) uint8_t smem_raw[];
    NmsSmem& sm = *reinterpret_cast<NmsSmem*>(smem_raw);
    const int t = threadIdx.x;
    const int n = min(raw_count, PD_MAX_CANDIDATES);
    int np2 = 64;
    while (np2 < n) np2 <<= 1;
    for (int q = t; q < np2; q += NMS_THREADS) {
        sm.key[q] = q < n ? sort_key(cs[q], ck[q]) : ~0ull;
        sm.sidx[q] = (uint16_t)q;
    }
    if (t == 0) sm.nkept = 0;
    __syncthreads();
    for (int k = 2; k <= np2; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int q = t; q < np2; q += NMS_THREADS) {
                const int p = q ^ jj;
                if (p > q) {
                    const unsigned long long a = sm.key[q], b = sm.key[p];
                    const bool up = (q & k) == 0;
                    if ((a > b) == up) {
                        sm.key[q] = b;
                        sm.key[p] = a;
                        const uint16_t ti = sm.sidx[q];
                        sm.sidx[q] = sm.sidx[p];
                        sm.sidx[p] = ti;
                    }
                }
            }
            __syncthreads();
        }
    }

    for (int c0 = 0; c0 < n; c0 += 64) {
        const int cn = min(64, n - c0);
        if (t < cn) {
            const int4 k = ck[sm.sidx[c0 + t]];
            sm.cbox[t] = window_box(g, k.x, k.y, k.z);
        }
        if (t < 64) {
            sm.supf[t] = 0u;
            sm.cmask[t] = 0ull;
        }
        __syncthreads();
        const int K = sm.nkept;
        const int q = t & 63, part = t >> 6;
        if (q < cn) {
            // against the boxes kept in earlier chunks: lane q of every wave
            // takes candidate q, the NMS_WAVES waves split the kept list, two
            // boxes per step
            const int4 cb = sm.cbox[q];
            bool hit = false;
            for (int kk = part; kk < K && !hit; kk += 2 * NMS_WAVES) {
                const int k2 = min(kk + NMS_WAVES, K - 1);
                const int4 a = sm.kbox[kk], b = sm.kbox[k2];
                hit = overlaps(cb, a) || overlaps(cb, b);
            }
            if (hit) sm.supf[q] = 1u;
            // in-chunk overlaps: candidate q against the later ones, four
            // columns per wave, merged into the candidate's mask by LDS OR
            unsigned long long m = 0;
#pragma unroll
            for (int u = 0; u < 64 / NMS_WAVES; ++u) {
                const int r = (64 / NMS_WAVES) * part + u;
                if (r > q && r < cn && overlaps(cb, sm.cbox[r])) m |= 1ull << r;
            }
            if (m) atomicOr(&sm.cmask[q], m);
        }
        __syncthreads();
        if (t < 64) {
            // wave 0 resolves the chunk: lane q holds candidate q's overlap mask;
            // the greedy walk over the chunk runs on the scalar unit with each
            // mask read from its lane, then the kept boxes are appended in
            // candidate order, one lane each
            const unsigned long long cm = q < cn ? sm.cmask[q] : 0ull;
            const unsigned long long sup = __ballot(q < cn && sm.supf[q] != 0u);
            unsigned long long alive = (cn == 64) ? ~0ull : ((1ull << cn) - 1);
            alive &= ~sup;
            const uint32_t cm_lo = (uint32_t)cm, cm_hi = (uint32_t)(cm >> 32);
            // the lowest alive candidate not yet visited is kept; it removes
            // the later ones it overlaps (its mask has only higher bits set)
            unsigned long long todo = alive;
            while (todo) {
                const int r = __builtin_ctzll(todo);
                const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(cm_lo, r);
                const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane(cm_hi, r);
                const unsigned long long mr = (unsigned long long)lo | ((unsigned long long)hi << 32);
                alive &= ~mr;
                todo &= alive & ~(1ull << r);
            }
            if ((alive >> q) & 1ull) {
                const int at = K + __popcll(alive & ((1ull << q) - 1ull));
                sm.kbox[at] = sm.cbox[q];
                sm.kpos[at] = (uint16_t)(c0 + q);
            }
            if (q == 0) sm.nkept = K + __popcll(alive);
        }
        __syncthreads();
    }

    const int K = sm.nkept;
    const int nout = min(K, cap);
    for (int q = t; q < nout; q += NMS_THREADS) {
        const int src = sm.sidx[sm.kpos[q]];
        const int4 k = ck[src];
        pd_box b;
        b.frame = frame;
        b.level = k.x;
        b.i = k.y;
        b.j = k.z;
        b.model = k.w;
        const int4 bx = sm.kbox[q];
        b.x0 = bx.x;
        b.y0 = bx.y;
        b.x1 = bx.z;
        b.y1 = bx.w;
        b.score = cs[src];
        b.score64 = c64 ? c64[src] : __longlong_as_double(0x7ff8000000000000LL);
        boxes[(size_t)frame * cap + q] = b;
    }
    if (t == 0) {
        pd_counts c;
        c.candidates = raw_count;
        c.kept = nout;
        c.overflow = (raw_count > PD_MAX_CANDIDATES || K > cap) ? 1 : 0;
        c.rescored = rescored;
        counts[frame] = c;
    }
}

__global__ void __launch_bounds__(NMS_THREADS) nms_table_kernel(const NmsGeom* __restrict__ geoms,
                                                        const int32_t* __restrict__ counters,
                                                        const float* __restrict__ cand_score,
                                                        const int4* __restrict__ cand_key,
                                                        const double* __restrict__ cand_s64,
                                                        const float* __restrict__ sel_score,
                                                        const int4* __restrict__ sel_key,
                                                        const double* __restrict__ sel_s64,
                                                        const int32_t* __restrict__ near_count,
                                                        pd_box* __restrict__ boxes, int cap,
                                                        pd_counts* __restrict__ counts) {
    const int f = blockIdx.x;
    const int n = counters[f];
    const float* cs;
    const int4* ck;
    const double* c64;
    if (n > PD_MAX_CANDIDATES) {  // the selected highest-scoring candidates
        const size_t o = (size_t)f * PD_MAX_CANDIDATES;
        cs = sel_score + o;
        ck = sel_key + o;
        c64 = sel_s64 ? sel_s64 + o : nullptr;
    } else {
        const size_t o = (size_t)geoms[f].cand_off;
        cs = cand_score + o;
        ck = cand_key + o;
        c64 = cand_s64 ? cand_s64 + o : nullptr;
    }
    nms_frame(geoms[f], f, n, cs, ck, c64, near_count ? near_count[f] : 0, boxes, cap, counts);
}

__global__ void __launch_bounds__(NMS_THREADS) nms_single_kernel(NmsGeom g, int n, const float* __restrict__ cs,
                                                         const int4* __restrict__ ck, pd_box* __restrict__ boxes,
                                                         int cap, pd_counts* __restrict__ counts) {
    nms_frame(g, 0, n, cs, ck, nullptr, 0, boxes, cap, counts);
}

constexpr size_t kNmsSmem = sizeof(NmsSmem);
static_assert(kNmsSmem <= 160 * 1024, "NMS scratch exceeds LDS");

}  // namespace

hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    zero_kernel<<<ceil_div(n, 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_compact(const LevelItem* items, const Tile* tiles, int n_tiles, int n_models,
                          const double* thresholds, float margin, int32_t* counters, float* cand_score,
                          int4* cand_key, double* cand_s64, int32_t* near_count, int4* near_key, int64_t near_cap,
                          int n_frames, const float* kth, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    compact_kernel<<<n_tiles, CP_THREADS, 0, s>>>(items, tiles, n_models, thresholds, margin, counters, cand_score, cand_key,
                                           cand_s64, near_count, near_key, near_cap, n_frames, kth);
    return hipGetLastError();
}

hipError_t launch_cand_select(const NmsGeom* geoms, int n_frames, const int32_t* counters, const float* cand_score,
                              const int4* cand_key, const double* cand_s64, float* sel_score, int4* sel_key,
                              double* sel_s64, hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    cand_select_kernel<<<n_frames, SEL_THREADS, 0, s>>>(geoms, counters, cand_score, cand_key, cand_s64, sel_score,
                                                        sel_key, sel_s64);
    return hipGetLastError();
}

hipError_t launch_nms_table(const NmsGeom* geoms, int n_frames, const int32_t* counters,
                            const float* cand_score, const int4* cand_key, const double* cand_s64,
                            const float* sel_score, const int4* sel_key, const double* sel_s64,
                            const int32_t* near_count, pd_box* boxes, int cap, pd_counts* counts, hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&nms_table_kernel),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kNmsSmem);
    if (attr != hipSuccess) return attr;
    nms_table_kernel<<<n_frames, NMS_THREADS, kNmsSmem, s>>>(geoms, counters, cand_score, cand_key, cand_s64,
                                                             sel_score, sel_key, sel_s64, near_count, boxes, cap,
                                                             counts);
    return hipGetLastError();
}

hipError_t launch_nms_single(const NmsGeom& g, int n, const float* cand_score, const int4* cand_key,
                             pd_box* boxes, int cap, pd_counts* counts, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&nms_single_kernel),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kNmsSmem);
    if (attr != hipSuccess) return attr;
    nms_single_kernel<<<1, NMS_THREADS, kNmsSmem, s>>>(g, n, cand_score, cand_key, boxes, cap, counts);
    return hipGetLastError();
}

}  // namespace pd
