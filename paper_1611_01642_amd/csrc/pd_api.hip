// C ABI of libpd: argument checks, pyramid planning, workspace layout and the
// launch sequence of the detection pipeline.  No allocation happens here:
// every device buffer comes from the caller.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pd_internal.h"

using namespace pd;

namespace {
thread_local std::string g_last_error;
}  // namespace

int pd::fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int pd::hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return PD_OK;
    return fail(PD_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

namespace {

constexpr int64_t kAlign = 256;
constexpr int FT_MIN_ROWS = 4, FT_MAX_ROWS = 32;  // feature strip heights accepted in tune_feat_rows
inline int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

bool check_params(const pd_params* p) {
    if (!p) return fail(PD_E_ARG, "params is NULL"), false;
    if (p->scale_den <= 0 || p->scale_num <= p->scale_den || p->scale_num > 1000000)
        return fail(PD_E_ARG, "scale must satisfy num > den > 0 (got %d/%d)", p->scale_num, p->scale_den),
               false;
    if (p->max_levels < 0) return fail(PD_E_ARG, "max_levels < 0"), false;
    if (!(p->clip > 0.0f) || !(p->eps > 0.0f) || !std::isfinite(p->clip) || !std::isfinite(p->eps))
        return fail(PD_E_ARG, "clip and eps must be positive"), false;
    if ((p->features & ~(PD_FEAT_HOG | PD_FEAT_LBP)) != 0 || (p->features & (PD_FEAT_HOG | PD_FEAT_LBP)) == 0)
        return fail(PD_E_ARG, "unknown feature flags 0x%x", p->features), false;
    if (p->precision != PD_PREC_F32 && p->precision != PD_PREC_BF16)
        return fail(PD_E_ARG, "unknown precision %d", p->precision), false;
    if (!(p->margin >= 0.0f) || !std::isfinite(p->margin)) return fail(PD_E_ARG, "margin must be >= 0"), false;
    if (p->tune_feat_rows != 0 && (p->tune_feat_rows < FT_MIN_ROWS || p->tune_feat_rows > FT_MAX_ROWS))
        return fail(PD_E_ARG, "tune_feat_rows must be 0 or in [%d, %d]", FT_MIN_ROWS, FT_MAX_ROWS), false;
    if (p->tune_score_rows != 0 && p->tune_score_rows != 4 && p->tune_score_rows != 8 && p->tune_score_rows != 16)
        return fail(PD_E_ARG, "tune_score_rows must be 0, 4, 8 or 16"), false;
    if (p->tune_grid < 0 || p->tune_grid > (1 << 20))
        return fail(PD_E_ARG, "tune_grid must be in [0, 2^20]"), false;
    if (p->prune_keep < 0) return fail(PD_E_ARG, "prune_keep must be >= 0"), false;
    if (p->prune_keep > 0 && !p->pruner) return fail(PD_E_ARG, "prune_keep > 0 needs the pruner weights"), false;
    if (p->prune_keep > 0 && p->features != (PD_FEAT_HOG | PD_FEAT_LBP))
        return fail(PD_E_ARG, "pruning needs HOG and LBP features"), false;
    return true;
}

// Tile and launch shapes from the tuning fields (0 selects the default).
Tuning tuning_of(const pd_params* p) {
    Tuning t;
    if (p->tune_feat_rows) t.feat_rows = p->tune_feat_rows;
    if (p->tune_score_rows) t.score_rows = p->tune_score_rows;
    t.grid = p->tune_grid;
    return t;
}

int check_image(const void* img, int w, int h, int pitch, const char* name) {
    if (w < 1 || h < 1 || w > PD_MAX_DIM || h > PD_MAX_DIM)
        return fail(PD_E_SIZE, "%s size %dx%d outside [1, %d]", name, w, h, PD_MAX_DIM);
    if (!img) return fail(PD_E_ARG, "%s is NULL", name);
    if (pitch < w) return fail(PD_E_ARG, "%s pitch %d < width %d", name, pitch, w);
    return PD_OK;
}

// Pinned host staging for the per-call tables.  A ring of slots, each reused
// only after the copy that last read it has finished.
struct Staging {
    struct Slot {
        void* host = nullptr;
        size_t size = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    };
    Slot slot[4];
    int next = 0;
    ~Staging() {
        for (auto& s : slot) {
            if (s.ev) (void)hipEventDestroy(s.ev);
            if (s.host) (void)hipHostFree(s.host);
        }
    }
};
thread_local Staging g_stage;

// Copies `bytes` of host tables to device `dst` through the next pinned
// staging slot (the slot is reused only after that copy has finished).
int stage_upload(const void* src, size_t bytes, void* dst, hipStream_t s) {
    Staging::Slot& slot = g_stage.slot[g_stage.next];
    g_stage.next = (g_stage.next + 1) % 4;
    if (slot.pending) {
        if (int rc = hip_status(hipEventSynchronize(slot.ev), "staging wait")) return rc;
        slot.pending = false;
    }
    if (!slot.ev) {
        if (int rc = hip_status(hipEventCreateWithFlags(&slot.ev, hipEventDisableTiming), "staging event")) return rc;
    }
    if (slot.size < bytes) {
        if (slot.host) (void)hipHostFree(slot.host);
        slot.host = nullptr;
        slot.size = 0;
        const size_t want = (size_t)align_up((int64_t)bytes, 1 << 16);
        if (int rc = hip_status(hipHostMalloc(&slot.host, want, hipHostMallocDefault), "staging alloc")) return rc;
        slot.size = want;
    }
    std::memcpy(slot.host, src, bytes);
    if (int rc = hip_status(hipMemcpyAsync(dst, slot.host, bytes, hipMemcpyHostToDevice, s), "table upload"))
        return rc;
    if (int rc = hip_status(hipEventRecord(slot.ev, s), "staging record")) return rc;
    slot.pending = true;
    return PD_OK;
}

// Workspace of the pruner calls: tables, weight copies, partials, then per
// map its activations (32 + 32 + 16 channels) and two 32-channel gradient
// buffers.
struct NetLayout {
    int n_tiles = 0;
    int64_t off_items = 0, off_tiles = 0, off_prep = 0, off_partial = 0, off_stats = 0, off_maps = 0, total = 0;
    std::vector<int64_t> map_off;
};

bool plan_net(const pd_net_map* maps, int n_maps, NetLayout& L) {
    L = NetLayout();
    for (int m = 0; m < n_maps; ++m) {
        const int wc = maps[m].cells_x, hc = maps[m].cells_y;
        if (wc < 1 || hc < 1 || wc > PD_MAX_DIM / PD_CELL || hc > PD_MAX_DIM / PD_CELL)
            return fail(PD_E_SIZE, "map %d size %dx%d outside [1, %d]", m, wc, hc, PD_MAX_DIM / PD_CELL), false;
        L.n_tiles += hc * ceil_div(wc, 64);
    }
    int64_t o = 0;
    L.off_items = o;
    o = align_up(o + (int64_t)n_maps * sizeof(NetItem), kAlign);
    L.off_tiles = o;
    o = align_up(o + (int64_t)L.n_tiles * sizeof(Tile), kAlign);
    L.off_prep = o;
    o = align_up(o + pruner_prep_floats() * 4, kAlign);
    L.off_partial = o;
    o = align_up(o + pruner_partial_floats(L.n_tiles) * 4, kAlign);
    L.off_stats = o;
    o = align_up(o + 16, kAlign);
    L.off_maps = o;
    for (int m = 0; m < n_maps; ++m) {
        L.map_off.push_back(o);
        o = align_up(o + (int64_t)(32 + 32 + 16 + 32 + 32) * maps[m].cells_x * maps[m].cells_y * 4, kAlign);
    }
    L.total = o;
    return true;
}

// Validates the maps and the workspace, uploads the tables.
int net_setup(const pd_net_map* maps, int n_maps, bool training, void* workspace, int64_t workspace_bytes,
              hipStream_t s, NetLayout& L) {
    if (!maps || n_maps < 1) return fail(PD_E_ARG, "maps is NULL or n_maps < 1");
    for (int m = 0; m < n_maps; ++m) {
        if (!maps[m].cellmap || !maps[m].logits) return fail(PD_E_ARG, "map %d: NULL cell map or logits", m);
        if (training && (!maps[m].labels || !maps[m].mask)) return fail(PD_E_ARG, "map %d: NULL labels or mask", m);
    }
    if (!plan_net(maps, n_maps, L)) return PD_E_SIZE;
    if (!workspace || workspace_bytes < L.total)
        return fail(PD_E_WORKSPACE, "workspace of %lld bytes, need %lld", (long long)workspace_bytes,
                    (long long)L.total);
    if ((uintptr_t)workspace & (kAlign - 1)) return fail(PD_E_ARG, "workspace must be 256-byte aligned");
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    std::vector<uint8_t> host((size_t)L.off_prep);
    NetItem* items = reinterpret_cast<NetItem*>(host.data() + L.off_items);
    Tile* tiles = reinterpret_cast<Tile*>(host.data() + L.off_tiles);
    int t = 0;
    for (int m = 0; m < n_maps; ++m) {
        const int wc = maps[m].cells_x, hc = maps[m].cells_y;
        const size_t plane = (size_t)wc * hc;
        NetItem& it = items[m];
        float* base = reinterpret_cast<float*>(ws + L.map_off[m]);
        it.buf[NET_X] = const_cast<float*>(maps[m].cellmap);
        it.buf[NET_A1] = base;
        it.buf[NET_A2] = base + 32 * plane;
        it.buf[NET_A3] = base + 64 * plane;
        it.buf[NET_GA] = base + 80 * plane;
        it.buf[NET_GB] = base + 112 * plane;
        it.logit = maps[m].logits;
        it.label = maps[m].labels;
        it.mask = maps[m].mask;
        it.wc = wc;
        it.hc = hc;
        for (int p = 0; p < hc; ++p)
            for (int tx = 0; tx < ceil_div(wc, 64); ++tx) tiles[t++] = Tile{m, p, tx, 0};
    }
    return stage_upload(host.data(), host.size(), ws, s);
}

// Unsigned big integer (32-bit limbs) for exact level sizes.
struct Big {
    std::vector<uint32_t> d{1};
    void mul(uint32_t m) {
        uint64_t carry = 0;
        for (auto& x : d) {
            const uint64_t v = (uint64_t)x * m + carry;
            x = (uint32_t)v;
            carry = v >> 32;
        }
        if (carry) d.push_back((uint32_t)carry);
    }
    // -1, 0, 1 for this <, ==, > o
    int cmp(const Big& o) const {
        size_t n = std::max(d.size(), o.d.size());
        for (size_t i = n; i-- > 0;) {
            const uint32_t a = i < d.size() ? d[i] : 0u, b = i < o.d.size() ? o.d[i] : 0u;
            if (a != b) return a < b ? -1 : 1;
        }
        return 0;
    }
};

// floor(a / b) for a result known to lie in [0, limit]: largest q with q*b <= a.
int big_floor_div(const Big& a, const Big& b, int limit) {
    int lo = 0, hi = limit;
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        Big t = b;
        t.mul((uint32_t)mid);
        if (t.cmp(a) <= 0) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Exact level sizes floor(n * den^k / num^k), kept while the window fits.
int plan_sizes(int w, int h, const pd_params* p, int (*wh)[2]) {
    Big num_k, den_w, den_h;
    den_w.mul((uint32_t)w);
    den_h.mul((uint32_t)h);
    int n = 0;
    for (int k = 0; k < PD_MAX_LEVELS; ++k) {
        const int wk = big_floor_div(den_w, num_k, w);
        const int hk = big_floor_div(den_h, num_k, h);
        if (wk < PD_WIN_W || hk < PD_WIN_H) break;
        wh[n][0] = wk;
        wh[n][1] = hk;
        ++n;
        if (p->max_levels && n >= p->max_levels) break;
        num_k.mul((uint32_t)p->scale_num);
        den_w.mul((uint32_t)p->scale_den);
        den_h.mul((uint32_t)p->scale_den);
    }
    return n;
}

void fill_level(pd_level& L, int w, int h) {
    std::memset(&L, 0, sizeof(L));
    L.w = w;
    L.h = h;
    L.pitch = (int)align_up(w, 16);
    L.cells_x = w / PD_CELL;
    L.cells_y = h / PD_CELL;
    L.blocks_x = L.cells_x - 1;
    L.blocks_y = L.cells_y - 1;
    L.win_x = L.cells_x - PD_WIN_CELLS_X + 1;
    L.win_y = L.cells_y - PD_WIN_CELLS_Y + 1;
}

void item_geometry(LevelItem& it, int w, int h) {
    it.w = w;
    it.h = h;
    it.wc = w / PD_CELL;
    it.hc = h / PD_CELL;
    it.wb = it.wc - 1;
    it.hb = it.hc - 1;
    it.nx = it.wc - PD_WIN_CELLS_X + 1;
    it.ny = it.hc - PD_WIN_CELLS_Y + 1;
}

// Layout of the pd_detect workspace; computed identically by the size query
// and by pd_detect.
struct DetectLayout {
    int n_items = 0;
    int n_rs = 0, n_ft = 0, n_sc = 0, n_cp = 0, n_pr = 0;  // tile table capacities
    bool bf16 = false;
    bool rowgemm = false;  // BF16, one model, HOG and LBP: the row-GEMM scoring kernel and its strip tiles
    bool prune = false;  // learned pruning: cell maps, network, top-K, tile filter
    int64_t off_kth = 0, off_kept = 0, off_prpack = 0;
    std::vector<int64_t> cm_off, a1_off, a2_off, lg_off;  // per item (pruning)
    int64_t off_items = 0, off_tiles = 0, off_geoms = 0, off_first = 0, off_counters = 0, off_cscore = 0,
            off_ckey = 0, off_c64 = 0, off_near_count = 0, off_near_key = 0, off_packed = 0, off_orient = 0;
    int64_t off_s32ctr = 0, off_s32pack = 0;  // FP32 scoring: band counters (zeroed with the others), packed weights
    int64_t off_sel_score = 0, off_sel_key = 0, off_sel_64 = 0;  // per frame, the top PD_MAX_CANDIDATES
    int64_t off_data = 0, total = 0;
    int64_t table_bytes = 0;  // bytes uploaded from the host (items .. geoms)
    int64_t n_windows = 0;    // windows of the batch: the candidate lists' and the near list's capacity
    std::vector<int64_t> cand_off;        // per frame: first entry of its candidate list
    std::vector<int> cand_cap;            // per frame: its window count
    std::vector<int> level_count;         // per frame
    std::vector<int> sizes;               // per item: w, h
    std::vector<int64_t> pyr_off, hog_off, lbp_off, sc_off;  // per item, from off_data
};

bool plan_detect(const pd_frame* frames, int n_frames, const pd_params* p, int n_models, DetectLayout& L) {
    L = DetectLayout();
    L.bf16 = p->precision == PD_PREC_BF16;
    L.rowgemm = L.bf16 && n_models == 1 && p->features == (PD_FEAT_HOG | PD_FEAT_LBP);
    L.prune = p->prune_keep > 0;
    L.level_count.resize(n_frames);
    int wh[PD_MAX_LEVELS][2];
    int64_t data = 0;
    for (int f = 0; f < n_frames; ++f) {
        const int w = frames[f].w, h = frames[f].h;
        if (w < 1 || h < 1 || w > PD_MAX_DIM || h > PD_MAX_DIM)
            return fail(PD_E_SIZE, "frame %d size %dx%d outside [1, %d]", f, w, h, PD_MAX_DIM), false;
        const int n = plan_sizes(w, h, p, wh);
        L.level_count[f] = n;
        L.cand_off.push_back(L.n_windows);
        int64_t frame_windows = 0;
        for (int k = 0; k < n; ++k) {
            LevelItem it{};
            item_geometry(it, wh[k][0], wh[k][1]);
            frame_windows += (int64_t)it.nx * it.ny;
            L.sizes.push_back(wh[k][0]);
            L.sizes.push_back(wh[k][1]);
            // level 0 is read from the frame itself when its rows are 8-byte
            // aligned, else copied here like the other levels
            L.pyr_off.push_back(data);
            data = align_up(data + (int64_t)align_up(it.w, 16) * it.h, kAlign);
            L.hog_off.push_back(data);
            data = align_up(data + (int64_t)PD_HOG_BLOCK * it.hb * it.wb * (L.bf16 ? 2 : 4), kAlign);
            L.lbp_off.push_back(data);
            data = align_up(data + (int64_t)PD_LBP_BINS * it.hc * it.wc, kAlign);
            L.sc_off.push_back(data);
            data = align_up(data + (int64_t)n_models * it.ny * it.nx * 4, kAlign);
            if (L.prune) {
                const int64_t cells = (int64_t)it.hc * it.wc;
                L.cm_off.push_back(data);
                data = align_up(data + cells * PR_CP1 * 2, kAlign);
                L.a1_off.push_back(data);
                data = align_up(data + cells * 32 * 2, kAlign);
                L.a2_off.push_back(data);
                data = align_up(data + cells * 32 * 2, kAlign);
                L.lg_off.push_back(data);
                data = align_up(data + cells * 4, kAlign);
                L.n_pr += pruner_mfma_tiles_y(it.hc) * ceil_div(it.wc, 64);
            }
            L.n_rs += resize_tiles_x(it.w) * resize_tiles_y(it.h);  // upper bound
            // table capacity for the finest tile shapes the tuning fields
            // allow, so the workspace size does not depend on them
            L.n_ft += (L.prune ? feat_tiles_x_cm(it.wc) : feat_tiles_x(it.wc)) * feat_tiles_y(it.hc, FT_MIN_ROWS);
            L.n_sc += !L.bf16    ? score32_band_capacity(it.nx, it.ny, it.wc)
                      : L.rowgemm ? ceil_div(it.nx, RG_TILE_C)
                                  : ceil_div(it.nx, MF_TILE_C) * ceil_div(it.ny, MF_TILE_R);
            L.n_cp += ceil_div(it.nx * it.ny, CP_N);
            ++L.n_items;
        }
        L.cand_cap.push_back((int)frame_windows);  // at most 2041 x 2033 x 51 levels < 2^31
        L.n_windows += frame_windows;
    }
    int64_t o = 0;
    L.off_items = o;
    o = align_up(o + (int64_t)L.n_items * sizeof(LevelItem), kAlign);
    L.off_tiles = o;
    o = align_up(o + (int64_t)(L.n_rs + L.n_ft + L.n_sc + L.n_cp + L.n_pr) * sizeof(Tile), kAlign);
    L.off_geoms = o;
    o = align_up(o + (int64_t)n_frames * sizeof(NmsGeom), kAlign);
    L.off_first = o;
    o = align_up(o + (int64_t)n_frames * 4, kAlign);
    L.table_bytes = o;
    L.off_counters = o;  // candidate counters, then near counters (zeroed together)
    o = align_up(o + (int64_t)n_frames * 4, kAlign);
    L.off_near_count = o;  // per-frame near counters + the dense list length (+ kept tiles)
    o = align_up(o + (int64_t)(n_frames + 2) * 4, kAlign);
    if (!L.bf16) {
        L.off_s32ctr = o;
        o = align_up(o + (int64_t)S32_COUNTERS * 4, kAlign);
    }
    // candidate lists: room for every window of every frame
    L.off_cscore = o;
    o = align_up(o + L.n_windows * 4, kAlign);
    L.off_ckey = o;
    o = align_up(o + L.n_windows * 16, kAlign);
    L.off_sel_score = o;
    o = align_up(o + (int64_t)n_frames * PD_MAX_CANDIDATES * 4, kAlign);
    L.off_sel_key = o;
    o = align_up(o + (int64_t)n_frames * PD_MAX_CANDIDATES * 16, kAlign);
    if (L.bf16) {
        L.off_c64 = o;
        o = align_up(o + L.n_windows * 8, kAlign);
        L.off_sel_64 = o;
        o = align_up(o + (int64_t)n_frames * PD_MAX_CANDIDATES * 8, kAlign);
        L.off_near_key = o;  // every window of the batch may be near
        o = align_up(o + L.n_windows * 16, kAlign);
        L.off_packed = o;
        o = align_up(o + (packed_weight_elems() + rowgemm_packed_elems()) * 2, kAlign);
        L.off_orient = o;
        o = align_up(o + ORIENT_BYTES, kAlign);
    }
    if (!L.bf16) {
        L.off_s32pack = o;
        o = align_up(o + score32_packed_floats(n_models) * 4, kAlign);
    }
    if (L.prune) {
        L.off_kth = o;
        o = align_up(o + (int64_t)n_frames * 4, kAlign);
        L.off_kept = o;
        o = align_up(o + (int64_t)L.n_sc * sizeof(Tile), kAlign);
        L.off_prpack = o;
        o = align_up(o + pruner_packed_bf16_elems() * 2, kAlign);
    }
    L.off_data = o;
    L.total = o + data;
    return true;
}


// Stage events of pd_detect (pd_profile_enable / pd_profile_read).
struct Profile {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<std::vector<hipEvent_t>> pending;  // PD_N_STAGES + 1 events per call
    double ms[PD_N_STAGES] = {};
    int64_t calls = 0;
    ~Profile() {
        for (auto& v : pending)
            for (auto e : v) (void)hipEventDestroy(e);
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};
thread_local Profile g_prof;

// The device's constant-rate clock into *slot (a stage boundary of a captured
// graph: a kernel node, ordered after the previous stage's kernels).
__global__ void stamp_kernel(unsigned long long* slot) {
    if (threadIdx.x == 0) *slot = __builtin_amdgcn_s_memrealtime();
}

// Records the boundary events of one pd_detect call (or nothing when off);
// with `stamps` set (graph captures), clock stamps instead of events.
struct StageMarks {
    std::vector<hipEvent_t> ev;
    unsigned long long* stamps = nullptr;
    explicit StageMarks(bool on) {
        if (!on) return;
        for (int k = 0; k <= PD_N_STAGES; ++k) {
            hipEvent_t e = nullptr;
            if (!g_prof.pool.empty()) {
                e = g_prof.pool.back();
                g_prof.pool.pop_back();
            } else if (hipEventCreate(&e) != hipSuccess) {
                e = nullptr;
            }
            ev.push_back(e);
        }
    }
    void mark(int k, hipStream_t s) {
        if (stamps) stamp_kernel<<<1, 64, 0, s>>>(stamps + k);
        if (!ev.empty() && ev[k]) (void)hipEventRecord(ev[k], s);
    }
    void commit() {
        if (!ev.empty()) g_prof.pending.push_back(std::move(ev));
    }
};

// Argument checks and workspace layout shared by pd_detect, pd_graph_create
// and pd_autotune.
int validate_detect(const pd_frame* frames, int n_frames, const float* weights, const float* bias, int n_models,
                    const pd_params* params, const double* thresholds, const void* workspace,
                    int64_t workspace_bytes, const pd_box* boxes, int cap, const pd_counts* counts,
                    DetectLayout& L) {
    if (!check_params(params)) return PD_E_ARG;
    if (!frames || n_frames < 1) return fail(PD_E_ARG, "frames is NULL or n_frames < 1");
    const int max_m = params->precision == PD_PREC_BF16 ? PD_MAX_MODELS_BF16 : PD_MAX_MODELS;
    if (n_models < 1 || n_models > max_m) return fail(PD_E_SIZE, "n_models outside [1, %d]", max_m);
    if (!weights || !bias || !thresholds || !counts || (cap > 0 && !boxes) || cap < 0)
        return fail(PD_E_ARG, "NULL pointer argument");
    for (int f = 0; f < n_frames; ++f) {
        if (int rc = check_image(frames[f].data, frames[f].w, frames[f].h, frames[f].pitch, "frame")) return rc;
    }
    if (!plan_detect(frames, n_frames, params, n_models, L)) return PD_E_SIZE;
    if (!workspace || workspace_bytes < L.total)
        return fail(PD_E_WORKSPACE, "workspace of %lld bytes, need %lld", (long long)workspace_bytes,
                    (long long)L.total);
    if ((uintptr_t)workspace & (kAlign - 1)) return fail(PD_E_ARG, "workspace must be 256-byte aligned");
    return PD_OK;
}

// Device-side view of one planned pd_detect call.
struct DetectRun {
    const LevelItem* items = nullptr;
    const Tile *t_rs = nullptr, *t_ft = nullptr, *t_sc = nullptr, *t_cp = nullptr;
    int nrs = 0, nft = 0, nsc = 0, ncp = 0;  // tiles in use
    XcdLists xs{};     // FP32 scoring: the band table's per-XCD lists
    int s32_grid = 0;  // and its launch width
    int32_t* s32_ctr = nullptr;
    float* s32_pack = nullptr;
    const NmsGeom* geoms = nullptr;
    const int32_t* first = nullptr;
    int32_t* counters = nullptr;
    int32_t* near_count = nullptr;
    float* cscore = nullptr;
    int4* ckey = nullptr;
    double* c64 = nullptr;
    float* sel_score = nullptr;  // per frame, its PD_MAX_CANDIDATES highest-scoring candidates
    int4* sel_key = nullptr;
    double* sel_64 = nullptr;
    int4* near_key = nullptr;
    int64_t near_cap = 0;
    uint16_t* packed = nullptr;
    double2* orient = nullptr;  // FP64 rescore's gradient table (BF16 precision)
    int n_zero = 0;  // counters + near counters (+ kept-tile count), cleared together
    const Tile* t_pr = nullptr;  // pruner conv tiles
    int npr = 0;
    float* kth = nullptr;        // per frame: K-th largest window logit
    Tile* kept = nullptr;        // score tiles that hold a kept window
    int32_t* kept_count = nullptr;
    uint16_t* prpack = nullptr;  // BF16 fragment-packed pruner weights
};

// Builds the level, tile and NMS tables of one call in host memory `stage`
// (L.table_bytes), laid out as they are uploaded to device memory `tbl`: the
// start of the workspace `ws` for pd_detect, a graph's own buffer for a
// captured graph.  Every other buffer is in `ws`.
void fill_tables(const pd_frame* frames, int n_frames, int n_models, const Tuning& tu, const DetectLayout& L,
                 uint8_t* ws, uint8_t* tbl, uint8_t* stage, DetectRun& R) {
    uint8_t* data = ws + L.off_data;
    std::memset(stage, 0, (size_t)L.table_bytes);
    LevelItem* items = reinterpret_cast<LevelItem*>(stage + L.off_items);
    Tile* tiles = reinterpret_cast<Tile*>(stage + L.off_tiles);
    NmsGeom* geoms = reinterpret_cast<NmsGeom*>(stage + L.off_geoms);
    int32_t* first = reinterpret_cast<int32_t*>(stage + L.off_first);
    Tile* t_rs = tiles;
    Tile* t_ft = t_rs + L.n_rs;
    Tile* t_sc = t_ft + L.n_ft;
    Tile* t_cp = t_sc + L.n_sc;
    Tile* t_pr = t_cp + L.n_cp;
    int q = 0, nrs = 0, nft = 0, nsc = 0, ncp = 0, npr = 0;
    for (int f = 0; f < n_frames; ++f) {
        geoms[f].n_levels = L.level_count[f];
        geoms[f].cand_off = L.cand_off[f];
        geoms[f].cand_cap = L.cand_cap[f];
        first[f] = q;
        for (int k = 0; k < L.level_count[f]; ++k, ++q) {
            LevelItem& it = items[q];
            item_geometry(it, L.sizes[2 * q], L.sizes[2 * q + 1]);
            it.src = frames[f].data;
            it.src_w = frames[f].w;
            it.src_h = frames[f].h;
            it.src_pitch = frames[f].pitch;
            const bool direct = k == 0 && (((uintptr_t)frames[f].data | (uintptr_t)frames[f].pitch) & 7) == 0;
            if (direct) {
                it.pyr = const_cast<uint8_t*>(frames[f].data);
                it.pitch = frames[f].pitch;
            } else {
                it.pyr = data + L.pyr_off[q];
                it.pitch = (int)align_up(it.w, 16);
            }
            if (L.bf16) it.hog16 = reinterpret_cast<uint16_t*>(data + L.hog_off[q]);
            else it.hog = reinterpret_cast<float*>(data + L.hog_off[q]);
            it.lbp = data + L.lbp_off[q];
            it.scores = reinterpret_cast<float*>(data + L.sc_off[q]);
            it.frame = f;
            it.level = k;
            it.cand_off = L.cand_off[f];
            it.cand_cap = L.cand_cap[f];
            geoms[f].wh[k][0] = it.w;
            geoms[f].wh[k][1] = it.h;
            if (!direct) {  // tiles of `rows` rows (at least RS_TY: within the capacity counted above)
                const int rows = resize_rows(it.w, it.h, it.src_w, it.src_h);
                for (int y = 0; y < it.h; y += rows)
                    for (int tx = 0; tx < resize_tiles_x(it.w); ++tx) t_rs[nrs++] = Tile{q, y, tx, rows};
            }
            const int fty = feat_tiles_y(it.hc, tu.feat_rows);
            if (L.prune) {
                for (int ty = 0; ty < fty; ++ty)
                    for (int tx = 0; tx < feat_tiles_x_cm(it.wc); ++tx) t_ft[nft++] = Tile{q, ty, tx, 0};
            } else {
                // full 64-lane strips of 63 block columns; the remaining columns
                // in narrower lane groups (pad = group width), each wave taking
                // 64 / width row chunks
                const int wb = it.wc - 1;
                const int full = wb > 0 ? wb / FT_BX : 0;
                const int tail = wb > 0 ? wb - full * FT_BX : 0;
                for (int ty = 0; ty < fty; ++ty)
                    for (int tx = 0; tx < full; ++tx) t_ft[nft++] = Tile{q, ty, tx, 64};
                if (tail > 0 || full == 0) {
                    int width = 2;
                    while (width - 1 < std::max(tail, 1)) width *= 2;
                    for (int ty = 0; ty < fty; ty += 64 / width) t_ft[nft++] = Tile{q, ty, full, width};
                }
            }
            if (L.prune) {
                it.cmap16 = reinterpret_cast<uint16_t*>(data + L.cm_off[q]);
                it.act1 = reinterpret_cast<uint16_t*>(data + L.a1_off[q]);
                it.act2 = reinterpret_cast<uint16_t*>(data + L.a2_off[q]);
                it.logit = reinterpret_cast<float*>(data + L.lg_off[q]);
                for (int ty = 0; ty < pruner_mfma_tiles_y(it.hc); ++ty)
                    for (int tx = 0; tx < ceil_div(it.wc, 64); ++tx) t_pr[npr++] = Tile{q, ty, tx, 0};
            }
            if (L.rowgemm) {
                for (int tx = 0; tx < ceil_div(it.nx, RG_TILE_C); ++tx) t_sc[nsc++] = Tile{q, 0, tx, 0};
            } else if (L.bf16) {
                for (int ty = 0; ty < ceil_div(it.ny, MF_TILE_R); ++ty)
                    for (int tx = 0; tx < ceil_div(it.nx, MF_TILE_C); ++tx) t_sc[nsc++] = Tile{q, ty, tx, 0};
            }
            for (int c = 0; c < ceil_div(it.nx * it.ny, CP_N); ++c) t_cp[ncp++] = Tile{q, 0, c, 0};
        }
    }
    if (nft > 1) {
        // feature strips longest first (cell rows walked; with the cell map,
        // one more above all but the first), so that the launch ends on its
        // shortest strips: a counting sort, stable within a length
        const int ch = tu.feat_rows;
        auto rows_of = [&](const Tile& t) {
            const int c0 = t.ty * ch;
            return std::max(0, std::min(c0 + ch, items[t.item].hc - 1) - c0 + 1);
        };
        std::vector<int> start(ch + 2, 0);
        for (int i = 0; i < nft; ++i) ++start[rows_of(t_ft[i])];
        for (int r = ch + 1, acc = 0; r >= 0; --r) {
            const int c = start[r];
            start[r] = acc;
            acc += c;
        }
        const std::vector<Tile> by_item(t_ft, t_ft + nft);
        for (const Tile& t : by_item) t_ft[start[rows_of(t)]++] = t;
    }
    if (!L.bf16) nsc = score32_bands(items, q, tu.score_rows, tu.grid, t_sc, &R.xs, &R.s32_grid);
    const Tile* d_tiles = reinterpret_cast<const Tile*>(tbl + L.off_tiles);
    R.items = reinterpret_cast<const LevelItem*>(tbl + L.off_items);
    R.t_rs = d_tiles;
    R.t_ft = d_tiles + L.n_rs;
    R.t_sc = d_tiles + L.n_rs + L.n_ft;
    R.t_cp = d_tiles + L.n_rs + L.n_ft + L.n_sc;
    R.nrs = nrs;
    R.nft = nft;
    R.nsc = nsc;
    R.ncp = ncp;
    R.geoms = reinterpret_cast<const NmsGeom*>(tbl + L.off_geoms);
    R.first = reinterpret_cast<const int32_t*>(tbl + L.off_first);
    R.counters = reinterpret_cast<int32_t*>(ws + L.off_counters);
    R.near_count = reinterpret_cast<int32_t*>(ws + L.off_near_count);
    R.cscore = reinterpret_cast<float*>(ws + L.off_cscore);
    R.ckey = reinterpret_cast<int4*>(ws + L.off_ckey);
    R.c64 = L.bf16 ? reinterpret_cast<double*>(ws + L.off_c64) : nullptr;
    R.sel_score = reinterpret_cast<float*>(ws + L.off_sel_score);
    R.sel_key = reinterpret_cast<int4*>(ws + L.off_sel_key);
    R.sel_64 = L.bf16 ? reinterpret_cast<double*>(ws + L.off_sel_64) : nullptr;
    R.near_key = L.bf16 ? reinterpret_cast<int4*>(ws + L.off_near_key) : nullptr;
    R.near_cap = L.bf16 ? L.n_windows : 0;
    R.packed = L.bf16 ? reinterpret_cast<uint16_t*>(ws + L.off_packed) : nullptr;
    R.orient = L.bf16 ? reinterpret_cast<double2*>(ws + L.off_orient) : nullptr;
    R.n_zero = (int)((L.off_cscore - L.off_counters) / 4);
    if (!L.bf16) {
        R.s32_ctr = reinterpret_cast<int32_t*>(ws + L.off_s32ctr);
        R.s32_pack = reinterpret_cast<float*>(ws + L.off_s32pack);
    }
    if (L.prune) {
        R.t_pr = d_tiles + L.n_rs + L.n_ft + L.n_sc + L.n_cp;
        R.npr = npr;
        R.kth = reinterpret_cast<float*>(ws + L.off_kth);
        R.kept = reinterpret_cast<Tile*>(ws + L.off_kept);
        R.kept_count = reinterpret_cast<int32_t*>(ws + L.off_near_count) + n_frames + 1;
        R.prpack = reinterpret_cast<uint16_t*>(ws + L.off_prpack);
    }
}

// The decision stages of one call, after the scores: threshold and
// compaction (kth: pruned keep set, or NULL; skipped where the scoring kernel
// took the decisions itself), FP64 rescoring of the windows within the margin
// (BF16), the selection of the highest-scoring candidates of an overlong
// list, NMS.
int enqueue_decide(const DetectRun& R, const DetectLayout& L, const float* weights, const float* bias, int n_models,
                   const pd_params* params, const double* thresholds, int n_frames, pd_box* boxes, int cap,
                   pd_counts* counts, StageMarks& marks, const float* kth, bool decided, hipStream_t s) {
    int rc;
    if (!decided &&
        (rc = hip_status(launch_compact(R.items, R.t_cp, R.ncp, n_models, thresholds, L.bf16 ? params->margin : 0.0f,
                                        R.counters, R.cscore, R.ckey, R.c64, R.near_count, R.near_key, R.near_cap,
                                        n_frames, kth, s),
                         "compact")))
        return rc;
    if (L.bf16 && (rc = hip_status(launch_rescore64(R.items, R.first, n_frames, R.near_count, R.near_key, weights,
                                                    bias, n_models, params->features, params->clip, params->eps,
                                                    thresholds, R.counters, R.cscore, R.ckey, R.c64, R.orient, s),
                                   "rescore")))
        return rc;
    if ((rc = hip_status(launch_cand_select(R.geoms, n_frames, R.counters, R.cscore, R.ckey, R.c64, R.sel_score,
                                            R.sel_key, R.sel_64, s),
                         "candidate select")))
        return rc;
    marks.mark(PD_STAGE_NMS, s);
    return hip_status(launch_nms_table(R.geoms, n_frames, R.counters, R.cscore, R.ckey, R.c64, R.sel_score, R.sel_key,
                                       R.sel_64, L.bf16 ? R.near_count : nullptr, boxes, cap, counts, s),
                      "nms");
}

// The kernel sequence of one call (tables already uploaded).  Only kernels are
// enqueued here, so the sequence can be captured into a graph.
int enqueue_detect(const DetectRun& R, const DetectLayout& L, const Tuning& tu, const float* weights,
                   const float* bias, int n_models, const pd_params* params, const double* thresholds, int n_frames,
                   pd_box* boxes, int cap, pd_counts* counts, StageMarks& marks, hipStream_t s) {
    int rc;
    marks.mark(PD_STAGE_ZERO, s);
    if ((rc = hip_status(launch_zero_i32(R.counters, R.n_zero, s), "zero"))) return rc;
    if (!L.bf16 && (rc = hip_status(launch_pack_score32(weights, n_models, R.s32_pack, s), "pack"))) return rc;
    if (L.bf16) {
        if ((rc = hip_status(launch_orient_table(R.orient, s), "gradient table"))) return rc;
        if ((rc = hip_status(launch_pack_weights(weights, n_models, R.packed, s), "pack"))) return rc;
        if ((rc = hip_status(launch_pack_rowgemm(weights, R.packed + packed_weight_elems(), s), "pack"))) return rc;
    }
    if (L.prune && (rc = hip_status(launch_pruner_pack_bf16(params->pruner, R.prpack, s), "pruner pack")))
        return rc;
    marks.mark(PD_STAGE_RESIZE, s);
    if ((rc = hip_status(launch_resize_table(R.items, R.t_rs, R.nrs, s), "resize"))) return rc;
    marks.mark(PD_STAGE_FEATURES, s);
    if (L.prune) {
        if ((rc = hip_status(launch_features_cellmap_table(R.items, R.t_ft, R.nft, params->clip, params->eps, tu, s),
                             "features + cell map")))
            return rc;
        marks.mark(PD_STAGE_SCORE, s);
        if ((rc = hip_status(launch_pruner_mfma(R.items, R.t_pr, R.npr, params->pruner, R.prpack, s), "pruner")))
            return rc;
        if ((rc = hip_status(launch_topk(R.items, R.first, R.geoms, n_frames, params->prune_keep, R.kth, s), "top-k")))
            return rc;
        if (!L.bf16) {
            // FP32: bands span whole rows of 16-column tiles, which nearly
            // always hold a kept window; the keep set acts in compaction
            rc = hip_status(launch_score32_table(R.items, R.t_sc, R.xs, R.s32_grid, R.s32_pack, bias, n_models,
                                                 params->features, tu.score_rows, R.s32_ctr, Decide32{}, s),
                            "score");
        } else if (L.rowgemm) {
            // one model: the row-GEMM kernel scores whole 64-column strips, which
            // nearly always hold a kept window; the keep set acts in compaction
            rc = hip_status(launch_rowgemm_table(R.items, R.t_sc, R.nsc, R.packed + packed_weight_elems(), bias,
                                                 tu.grid, s),
                            "bf16 score");
        } else {
            rc = hip_status(launch_tile_filter(R.items, R.t_sc, R.nsc, MF_TILE_R, MF_TILE_C, R.kth, R.kept,
                                               R.kept_count, s),
                            "tile filter");
            if (!rc)
                rc = hip_status(launch_mfma_table(R.items, R.kept, R.nsc, R.packed, bias, n_models, params->features,
                                                  tu.grid, s, R.kept_count),
                                "bf16 score");
        }
        if (rc) return rc;
        marks.mark(PD_STAGE_COMPACT, s);
        return enqueue_decide(R, L, weights, bias, n_models, params, thresholds, n_frames, boxes, cap, counts, marks,
                              R.kth, false, s);
    }
    if ((rc = hip_status(launch_features_table(R.items, R.t_ft, R.nft, params->features, params->clip, params->eps,
                                               tu, s),
                         "features")))
        return rc;
    marks.mark(PD_STAGE_SCORE, s);
    bool decided = false;
    if (L.rowgemm) {
        if ((rc = hip_status(launch_rowgemm_table(R.items, R.t_sc, R.nsc, R.packed + packed_weight_elems(), bias,
                                                  tu.grid, s),
                             "bf16 score")))
            return rc;
    } else if (L.bf16) {
        if ((rc = hip_status(launch_mfma_table(R.items, R.t_sc, R.nsc, R.packed, bias, n_models, params->features,
                                               tu.grid, s),
                             "bf16 score")))
            return rc;
    } else {
        // FP32 with one model: each window's score is final when stored, and
        // the scoring kernel appends the candidates itself (bands of 4 or 8
        // window rows per wave: the shapes with room for it)
        decided = n_models == 1 && tu.score_rows != 16;
        const Decide32 dec = decided ? Decide32{thresholds, R.counters, R.cscore, R.ckey} : Decide32{};
        if ((rc = hip_status(launch_score32_table(R.items, R.t_sc, R.xs, R.s32_grid, R.s32_pack, bias, n_models,
                                                  params->features, tu.score_rows, R.s32_ctr, dec, s),
                             "score")))
            return rc;
    }
    marks.mark(PD_STAGE_COMPACT, s);
    return enqueue_decide(R, L, weights, bias, n_models, params, thresholds, n_frames, boxes, cap, counts, marks,
                          nullptr, decided, s);
}

}  // namespace

bool pd::profiling_on() { return g_prof.on; }

extern "C" {

int pd_profile_enable(int on) {
    g_prof.on = on != 0;
    return PD_OK;
}

int pd_profile_read(double* ms, int64_t* calls, int reset) {
    if (!ms || !calls) return fail(PD_E_ARG, "NULL output");
    for (auto& v : g_prof.pending) {
        bool ok = true;
        for (auto e : v) ok = ok && e;
        if (ok) {
            if (int rc = hip_status(hipEventSynchronize(v.back()), "profile wait")) return rc;
            for (int k = 0; k < PD_N_STAGES; ++k) {
                float t = 0.0f;
                if (hipEventElapsedTime(&t, v[k], v[k + 1]) == hipSuccess) g_prof.ms[k] += t;
            }
            ++g_prof.calls;
        }
        for (auto e : v)
            if (e) g_prof.pool.push_back(e);
    }
    g_prof.pending.clear();
    for (int k = 0; k < PD_N_STAGES; ++k) ms[k] = g_prof.ms[k];
    *calls = g_prof.calls;
    if (reset) {
        for (double& v : g_prof.ms) v = 0.0;
        g_prof.calls = 0;
    }
    return PD_OK;
}


void pd_params_default(pd_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->scale_num = 11;
    p->scale_den = 10;
    p->max_levels = 0;
    p->clip = 0.2f;
    p->eps = 1e-3f;
    p->features = PD_FEAT_HOG | PD_FEAT_LBP;
    p->precision = PD_PREC_F32;
    p->margin = 0.05f;
}

const char* pd_strerror(int code) {
    switch (code) {
        case PD_OK: return "ok";
        case PD_E_ARG: return "invalid argument";
        case PD_E_SIZE: return "invalid size";
        case PD_E_WORKSPACE: return "workspace missing or too small";
        case PD_E_HIP: return "HIP error";
        case PD_E_OVERFLOW: return "results truncated";
        case PD_E_IO: return "file error";
        default: return "unknown error";
    }
}

const char* pd_last_error(void) { return g_last_error.c_str(); }

const char* pd_version(void) { return "pd 0.1 gfx950"; }

int pd_plan_pyramid(int w, int h, const pd_params* params, pd_level* levels, int cap, int* n_levels,
                    int64_t* bytes) {
    if (!check_params(params)) return PD_E_ARG;
    if (!n_levels || !bytes || (cap > 0 && !levels) || cap < 0) return fail(PD_E_ARG, "null output");
    if (w < 1 || h < 1 || w > PD_MAX_DIM || h > PD_MAX_DIM)
        return fail(PD_E_SIZE, "image size %dx%d outside [1, %d]", w, h, PD_MAX_DIM);
    int wh[PD_MAX_LEVELS][2];
    const int n = plan_sizes(w, h, params, wh);
    int64_t off = 0;
    for (int k = 0; k < n; ++k) {
        pd_level L;
        fill_level(L, wh[k][0], wh[k][1]);
        L.offset = off;
        off = align_up(off + (int64_t)L.pitch * L.h, kAlign);
        if (k < cap) levels[k] = L;
    }
    *n_levels = n;
    *bytes = off;
    return PD_OK;
}

int pd_build_pyramid(const uint8_t* img, int w, int h, int pitch, const pd_level* levels, int n, uint8_t* pyr,
                     void* stream) {
    if (int rc = check_image(img, w, h, pitch, "img")) return rc;
    if (n < 0 || n > PD_MAX_LEVELS) return fail(PD_E_SIZE, "level count %d outside [0, %d]", n, PD_MAX_LEVELS);
    if (n == 0) return PD_OK;
    if (!levels || !pyr) return fail(PD_E_ARG, "levels or pyr is NULL");
    LevelItem items[PD_MAX_LEVELS];
    for (int k = 0; k < n; ++k) {
        const pd_level& L = levels[k];
        if (L.w < 1 || L.h < 1 || L.w > w || L.h > h || L.pitch < L.w || (L.pitch & 15) || (L.offset & 255))
            return fail(PD_E_ARG, "level %d is not a valid plan entry", k);
        items[k] = LevelItem{};
        items[k].src = img;
        items[k].src_w = w;
        items[k].src_h = h;
        items[k].src_pitch = pitch;
        items[k].pyr = pyr + L.offset;
        items[k].w = L.w;
        items[k].h = L.h;
        items[k].pitch = L.pitch;
    }
    return hip_status(launch_resize_single(items, n, (hipStream_t)stream), "pyramid launch");
}

int pd_lbp_codes(const uint8_t* lvl, int w, int h, int pitch, uint8_t* codes, int codes_pitch, void* stream) {
    if (int rc = check_image(lvl, w, h, pitch, "level")) return rc;
    if (!codes || codes_pitch < w) return fail(PD_E_ARG, "codes is NULL or its pitch < width");
    return hip_status(launch_lbp_codes(lvl, w, h, pitch, codes, codes_pitch, (hipStream_t)stream), "lbp codes");
}

int pd_features(const uint8_t* lvl, int w, int h, int pitch, const pd_params* params, float* blocks,
                uint16_t* blocks_bf16, uint8_t* cell_hist, void* stream) {
    if (int rc = check_image(lvl, w, h, pitch, "level")) return rc;
    if (!check_params(params)) return PD_E_ARG;
    if (blocks && blocks_bf16) return fail(PD_E_ARG, "give either FP32 or BF16 HOG output, not both");
    int feat = 0;
    if (blocks || blocks_bf16) feat |= PD_FEAT_HOG;
    if (cell_hist) feat |= PD_FEAT_LBP;
    if (!feat) return fail(PD_E_ARG, "all outputs are NULL");
    LevelItem it{};
    item_geometry(it, w, h);
    it.pyr = const_cast<uint8_t*>(lvl);
    it.pitch = pitch;
    it.hog = blocks;
    it.hog16 = blocks_bf16;
    it.lbp = cell_hist;
    if (it.hc < 1 || it.wc < 1) return PD_OK;  // no whole cell: nothing to write
    if ((feat & PD_FEAT_HOG) && (it.hb < 1 || it.wb < 1)) feat &= ~PD_FEAT_HOG;
    if (!feat) return PD_OK;
    return hip_status(launch_features_single(it, feat, params->clip, params->eps, (hipStream_t)stream),
                      "features launch");
}

int pd_features_cellmap(const uint8_t* lvl, int w, int h, int pitch, const pd_params* params, float* blocks,
                        uint8_t* cell_hist, float* cellmap, void* stream) {
    if (int rc = check_image(lvl, w, h, pitch, "level")) return rc;
    if (!check_params(params)) return PD_E_ARG;
    if (!blocks || !cell_hist || !cellmap) return fail(PD_E_ARG, "NULL output");
    LevelItem it{};
    item_geometry(it, w, h);
    if (it.hb < 1 || it.wb < 1) return fail(PD_E_SIZE, "level %dx%d has no 16x16 block", w, h);
    it.pyr = const_cast<uint8_t*>(lvl);
    it.pitch = pitch;
    it.hog = blocks;
    it.lbp = cell_hist;
    it.cmap = cellmap;
    return hip_status(launch_features_cellmap_single(it, params->clip, params->eps, (hipStream_t)stream),
                      "cell map launch");
}

int64_t pd_pruner_workspace_bytes(const pd_net_map* maps, int n_maps) {
    if (!maps || n_maps < 1) return fail(PD_E_ARG, "maps is NULL or n_maps < 1");
    NetLayout L;
    if (!plan_net(maps, n_maps, L)) return PD_E_SIZE;
    return L.total;
}

int pd_pruner_forward(const pd_net_map* maps, int n_maps, const float* params, void* workspace,
                      int64_t workspace_bytes, void* stream) {
    if (!params) return fail(PD_E_ARG, "params is NULL");
    hipStream_t s = (hipStream_t)stream;
    NetLayout L;
    if (int rc = net_setup(maps, n_maps, false, workspace, workspace_bytes, s, L)) return rc;
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    float* prep = reinterpret_cast<float*>(ws + L.off_prep);
    if (int rc = hip_status(launch_pruner_prep(params, prep, s), "pruner weights")) return rc;
    return hip_status(launch_pruner_forward(reinterpret_cast<const NetItem*>(ws + L.off_items),
                                            reinterpret_cast<const Tile*>(ws + L.off_tiles), L.n_tiles, params, prep,
                                            false, s),
                      "pruner forward");
}

int pd_pruner_gradient(const pd_net_map* maps, int n_maps, const float* params, float pos_weight, float* grad,
                       double* stats, void* workspace, int64_t workspace_bytes, void* stream) {
    if (!params || !grad || !stats) return fail(PD_E_ARG, "NULL pointer argument");
    if (!(pos_weight > 0.0f) || !std::isfinite(pos_weight)) return fail(PD_E_ARG, "pos_weight must be > 0");
    hipStream_t s = (hipStream_t)stream;
    NetLayout L;
    if (int rc = net_setup(maps, n_maps, true, workspace, workspace_bytes, s, L)) return rc;
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    const NetItem* items = reinterpret_cast<const NetItem*>(ws + L.off_items);
    const Tile* tiles = reinterpret_cast<const Tile*>(ws + L.off_tiles);
    float* prep = reinterpret_cast<float*>(ws + L.off_prep);
    int rc;
    if ((rc = hip_status(launch_pruner_prep(params, prep, s), "pruner weights"))) return rc;
    if ((rc = hip_status(launch_pruner_forward(items, tiles, L.n_tiles, params, prep, true, s), "pruner forward")))
        return rc;
    return hip_status(launch_pruner_backward(items, tiles, L.n_tiles, params, prep, pos_weight, grad, stats,
                                             reinterpret_cast<float*>(ws + L.off_partial), s),
                      "pruner backward");
}

int pd_adam_step(float* params, const float* grad, float* m, float* v, int n, int step, float lr, float beta1,
                 float beta2, float eps, void* stream) {
    if (!params || !grad || !m || !v) return fail(PD_E_ARG, "NULL pointer argument");
    if (n < 1 || step < 1) return fail(PD_E_SIZE, "n and step must be >= 1");
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(PD_E_ARG, "lr > 0, beta1 and beta2 in [0, 1), eps > 0 required");
    return hip_status(launch_adam(params, grad, m, v, n, step, lr, beta1, beta2, eps, (hipStream_t)stream), "adam");
}

int pd_window_labels(const float* scores, int win_x, int win_y, int cells_x, int cells_y, const double* threshold,
                     float* labels, float* mask, void* stream) {
    if (!scores || !threshold || !labels || !mask) return fail(PD_E_ARG, "NULL pointer argument");
    if (win_x < 1 || win_y < 1 || win_x + PD_WIN_CELLS_X - 1 != cells_x || win_y + PD_WIN_CELLS_Y - 1 != cells_y)
        return fail(PD_E_SIZE, "window grid %dx%d does not match cells %dx%d", win_x, win_y, cells_x, cells_y);
    return hip_status(launch_window_labels(scores, win_x, win_y, cells_x, cells_y, threshold, labels, mask,
                                           (hipStream_t)stream),
                      "labels");
}

// Workspace of pd_pruner_logits_bf16 for one w x h level.
struct LogitsLayout {
    int n_tiles = 0;
    int64_t off_item = 0, off_tiles = 0, off_packed = 0, off_hog = 0, off_lbp = 0, off_cmap = 0, off_a1 = 0,
            off_a2 = 0, total = 0;
};

LogitsLayout plan_logits(int w, int h) {
    LogitsLayout L;
    LevelItem it{};
    item_geometry(it, w, h);
    L.n_tiles = pruner_mfma_tiles_y(it.hc) * ceil_div(it.wc, 64);
    const int64_t cells = (int64_t)it.hc * it.wc;
    int64_t o = 0;
    L.off_item = o;
    o = align_up(o + (int64_t)sizeof(LevelItem), kAlign);
    L.off_tiles = o;
    o = align_up(o + (int64_t)L.n_tiles * sizeof(Tile), kAlign);
    L.off_packed = o;
    o = align_up(o + pruner_packed_bf16_elems() * 2, kAlign);
    L.off_hog = o;
    o = align_up(o + (int64_t)PD_HOG_BLOCK * std::max(it.hb, 0) * std::max(it.wb, 0) * 4, kAlign);
    L.off_lbp = o;
    o = align_up(o + (int64_t)PD_LBP_BINS * cells, kAlign);
    L.off_cmap = o;
    o = align_up(o + cells * PR_CP1 * 2, kAlign);
    L.off_a1 = o;
    o = align_up(o + cells * 32 * 2, kAlign);
    L.off_a2 = o;
    o = align_up(o + cells * 32 * 2, kAlign);
    L.total = o;
    return L;
}

int64_t pd_pruner_logits_bf16_workspace_bytes(int w, int h) {
    if (w < PD_WIN_W || h < PD_WIN_H || w > PD_MAX_DIM || h > PD_MAX_DIM)
        return fail(PD_E_SIZE, "level %dx%d outside [64x128, %d]", w, h, PD_MAX_DIM);
    return plan_logits(w, h).total;
}

int pd_pruner_logits_bf16(const uint8_t* lvl, int w, int h, int pitch, const pd_params* params,
                          const float* pruner, float* logits, void* workspace, int64_t workspace_bytes,
                          void* stream) {
    if (int rc = check_image(lvl, w, h, pitch, "level")) return rc;
    if (!check_params(params)) return PD_E_ARG;
    if (w < PD_WIN_W || h < PD_WIN_H) return fail(PD_E_SIZE, "level %dx%d smaller than a window", w, h);
    if (!pruner || !logits) return fail(PD_E_ARG, "NULL pointer argument");
    const LogitsLayout L = plan_logits(w, h);
    if (!workspace || workspace_bytes < L.total)
        return fail(PD_E_WORKSPACE, "workspace of %lld bytes, need %lld", (long long)workspace_bytes,
                    (long long)L.total);
    if ((uintptr_t)workspace & (kAlign - 1)) return fail(PD_E_ARG, "workspace must be 256-byte aligned");
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint8_t> host((size_t)L.off_packed);
    LevelItem& it = *reinterpret_cast<LevelItem*>(host.data() + L.off_item);
    item_geometry(it, w, h);
    it.pyr = const_cast<uint8_t*>(lvl);
    it.pitch = pitch;
    it.hog = reinterpret_cast<float*>(ws + L.off_hog);
    it.lbp = ws + L.off_lbp;
    it.cmap16 = reinterpret_cast<uint16_t*>(ws + L.off_cmap);
    it.act1 = reinterpret_cast<uint16_t*>(ws + L.off_a1);
    it.act2 = reinterpret_cast<uint16_t*>(ws + L.off_a2);
    it.logit = logits;
    Tile* tiles = reinterpret_cast<Tile*>(host.data() + L.off_tiles);
    int t = 0;
    for (int ty = 0; ty < pruner_mfma_tiles_y(it.hc); ++ty)
        for (int tx = 0; tx < ceil_div(it.wc, 64); ++tx) tiles[t++] = Tile{0, ty, tx, 0};
    int rc;
    if ((rc = stage_upload(host.data(), host.size(), ws, s))) return rc;
    uint16_t* packed = reinterpret_cast<uint16_t*>(ws + L.off_packed);
    if ((rc = hip_status(launch_pruner_pack_bf16(pruner, packed, s), "pruner pack"))) return rc;
    if ((rc = hip_status(launch_features_cellmap_single(it, params->clip, params->eps, s), "cell map"))) return rc;
    return hip_status(launch_pruner_mfma(reinterpret_cast<const LevelItem*>(ws + L.off_item),
                                         reinterpret_cast<const Tile*>(ws + L.off_tiles), L.n_tiles, pruner, packed,
                                         s),
                      "pruner mfma");
}

int pd_lbp(const uint8_t* lvl, int w, int h, int pitch, uint8_t* cell_hist, void* stream) {
    if (!cell_hist) return fail(PD_E_ARG, "cell_hist is NULL");
    pd_params p;
    pd_params_default(&p);
    return pd_features(lvl, w, h, pitch, &p, nullptr, nullptr, cell_hist, stream);
}

int pd_hog(const uint8_t* lvl, int w, int h, int pitch, const pd_params* params, float* blocks, void* stream) {
    if (!blocks) return fail(PD_E_ARG, "blocks is NULL");
    return pd_features(lvl, w, h, pitch, params, blocks, nullptr, nullptr, stream);
}

int pd_score_windows(const float* blocks, const uint8_t* cells, int cells_x, int cells_y, const float* weights,
                     const float* bias, int n_models, float* scores, void* stream) {
    if (cells_x < PD_WIN_CELLS_X || cells_y < PD_WIN_CELLS_Y || cells_x > PD_MAX_DIM / PD_CELL ||
        cells_y > PD_MAX_DIM / PD_CELL)
        return fail(PD_E_SIZE, "cell grid %dx%d cannot hold a window", cells_x, cells_y);
    if (n_models < 1 || n_models > PD_MAX_MODELS) return fail(PD_E_SIZE, "n_models %d outside [1, %d]", n_models, PD_MAX_MODELS);
    if (!blocks || !cells || !weights || !bias || !scores) return fail(PD_E_ARG, "NULL pointer argument");
    LevelItem it{};
    item_geometry(it, cells_x * PD_CELL, cells_y * PD_CELL);
    it.hog = const_cast<float*>(blocks);
    it.lbp = const_cast<uint8_t*>(cells);
    it.scores = scores;
    return hip_status(launch_score_single(it, weights, bias, n_models, PD_FEAT_HOG | PD_FEAT_LBP,
                                          (hipStream_t)stream),
                      "score launch");
}

int pd_lbp_naive(const uint8_t* codes, int w, int h, int codes_pitch, uint32_t* cell_hist, void* stream) {
    if (int rc = check_image(codes, w, h, codes_pitch, "codes")) return rc;
    if (!cell_hist) return fail(PD_E_ARG, "cell_hist is NULL");
    return hip_status(launch_lbp_naive(codes, codes_pitch, w / PD_CELL, h / PD_CELL, cell_hist, (hipStream_t)stream),
                      "lbp naive launch");
}

int pd_lbp_scatter(const uint8_t* codes, int w, int h, int codes_pitch, uint32_t* cell_hist, void* stream) {
    if (int rc = check_image(codes, w, h, codes_pitch, "codes")) return rc;
    if (!cell_hist) return fail(PD_E_ARG, "cell_hist is NULL");
    return hip_status(launch_lbp_scatter(codes, codes_pitch, w / PD_CELL, h / PD_CELL, cell_hist, (hipStream_t)stream),
                      "lbp scatter launch");
}

int pd_hog_global(const uint8_t* lvl, int w, int h, int pitch, const pd_params* params, float* grad, float* blocks,
                  void* stream) {
    if (int rc = check_image(lvl, w, h, pitch, "level")) return rc;
    if (!check_params(params)) return PD_E_ARG;
    if (!grad || !blocks) return fail(PD_E_ARG, "grad or blocks is NULL");
    return hip_status(launch_hog_global(lvl, w, h, pitch, params->clip, params->eps, grad, blocks, (hipStream_t)stream),
                      "hog global launch");
}

// Shared checks of the two baseline scoring entry points.
static int check_score_args(const float* blocks, const uint8_t* cells, int cells_x, int cells_y, const float* weights,
                            const float* bias, int n_models, const float* scores) {
    if (cells_x < PD_WIN_CELLS_X || cells_y < PD_WIN_CELLS_Y || cells_x > PD_MAX_DIM / PD_CELL ||
        cells_y > PD_MAX_DIM / PD_CELL)
        return fail(PD_E_SIZE, "cell grid %dx%d cannot hold a window", cells_x, cells_y);
    if (n_models < 1 || n_models > PD_MAX_MODELS)
        return fail(PD_E_SIZE, "n_models %d outside [1, %d]", n_models, PD_MAX_MODELS);
    if (!blocks || !cells || !weights || !bias || !scores) return fail(PD_E_ARG, "NULL pointer argument");
    return PD_OK;
}

int pd_score_windows_naive(const float* blocks, const uint8_t* cells, int cells_x, int cells_y, const float* weights,
                           const float* bias, int n_models, float* scores, void* stream) {
    if (int rc = check_score_args(blocks, cells, cells_x, cells_y, weights, bias, n_models, scores)) return rc;
    return hip_status(launch_svm_naive(blocks, cells, cells_x, cells_y, weights, bias, n_models, scores,
                                       (hipStream_t)stream),
                      "svm naive launch");
}

int pd_score_windows_wave(const float* blocks, const uint8_t* cells, int cells_x, int cells_y, const float* weights,
                          const float* bias, int n_models, float* scores, void* stream) {
    if (int rc = check_score_args(blocks, cells, cells_x, cells_y, weights, bias, n_models, scores)) return rc;
    return hip_status(launch_svm_wave(blocks, cells, cells_x, cells_y, weights, bias, n_models, scores,
                                      (hipStream_t)stream),
                      "svm wave launch");
}

int pd_lbp_blocks(const uint8_t* cells, int n, int hc, int wc, uint16_t* blocks, void* stream) {
    if (n < 1 || hc < 2 || wc < 2 || hc > PD_MAX_DIM / PD_CELL || wc > PD_MAX_DIM / PD_CELL ||
        (int64_t)n * PD_LBP_BINS * hc > INT32_MAX)
        return fail(PD_E_SIZE, "cell grid %dx%d x %d images has no block", wc, hc, n);
    if (!cells || !blocks) return fail(PD_E_ARG, "NULL pointer argument");
    return hip_status(launch_lbp_blocks(cells, n, hc, wc, blocks, (hipStream_t)stream), "lbp blocks launch");
}

int pd_fold_lbp_weights(const float* wb, int n_models, float* w, void* stream) {
    if (n_models < 1 || n_models > PD_MAX_MODELS) return fail(PD_E_SIZE, "n_models %d outside [1, %d]", n_models, PD_MAX_MODELS);
    if (!wb || !w) return fail(PD_E_ARG, "NULL pointer argument");
    return hip_status(launch_fold_lbp_weights(wb, n_models, w, (hipStream_t)stream), "fold launch");
}

int64_t pd_packed_models_bytes(void) { return (packed_weight_elems() + rowgemm_packed_elems()) * 2; }

int pd_pack_models(const float* weights, int n_models, uint16_t* packed, void* stream) {
    if (n_models < 1 || n_models > PD_MAX_MODELS_BF16)
        return fail(PD_E_SIZE, "n_models %d outside [1, %d]", n_models, PD_MAX_MODELS_BF16);
    if (!weights || !packed) return fail(PD_E_ARG, "NULL pointer argument");
    if (int rc = hip_status(launch_pack_weights(weights, n_models, packed, (hipStream_t)stream), "pack launch"))
        return rc;
    return hip_status(launch_pack_rowgemm(weights, packed + packed_weight_elems(), (hipStream_t)stream),
                      "pack launch");
}

int pd_score_windows_bf16(const uint16_t* blocks_bf16, const uint8_t* cells, int cells_x, int cells_y,
                          const uint16_t* packed, const float* bias, int n_models, float* scores, void* stream) {
    if (cells_x < PD_WIN_CELLS_X || cells_y < PD_WIN_CELLS_Y || cells_x > PD_MAX_DIM / PD_CELL ||
        cells_y > PD_MAX_DIM / PD_CELL)
        return fail(PD_E_SIZE, "cell grid %dx%d cannot hold a window", cells_x, cells_y);
    if (n_models < 1 || n_models > PD_MAX_MODELS_BF16)
        return fail(PD_E_SIZE, "n_models %d outside [1, %d]", n_models, PD_MAX_MODELS_BF16);
    if (!blocks_bf16 || !cells || !packed || !bias || !scores) return fail(PD_E_ARG, "NULL pointer argument");
    LevelItem it{};
    item_geometry(it, cells_x * PD_CELL, cells_y * PD_CELL);
    it.hog16 = const_cast<uint16_t*>(blocks_bf16);
    it.lbp = const_cast<uint8_t*>(cells);
    it.scores = scores;
    if (n_models == 1)
        return hip_status(launch_rowgemm_single(it, packed + packed_weight_elems(), bias, (hipStream_t)stream),
                          "bf16 score launch");
    return hip_status(launch_mfma_single(it, packed, bias, n_models, PD_FEAT_HOG | PD_FEAT_LBP, (hipStream_t)stream),
                      "bf16 score launch");
}

int64_t pd_detect_workspace_bytes(const pd_frame* frames, int n_frames, const pd_params* params, int n_models) {
    if (!check_params(params)) return PD_E_ARG;
    if (!frames || n_frames < 1) return fail(PD_E_ARG, "frames is NULL or n_frames < 1");
    const int max_m = params->precision == PD_PREC_BF16 ? PD_MAX_MODELS_BF16 : PD_MAX_MODELS;
    if (n_models < 1 || n_models > max_m) return fail(PD_E_SIZE, "n_models outside [1, %d]", max_m);
    DetectLayout L;
    if (!plan_detect(frames, n_frames, params, n_models, L)) return PD_E_SIZE;
    return L.total;
}

int pd_detect(const pd_frame* frames, int n_frames, const float* weights, const float* bias, int n_models,
              const pd_params* params, const double* thresholds, void* workspace, int64_t workspace_bytes,
              pd_box* boxes, int cap, pd_counts* counts, void* stream) {
    DetectLayout L;
    if (int rc = validate_detect(frames, n_frames, weights, bias, n_models, params, thresholds, workspace,
                                 workspace_bytes, boxes, cap, counts, L))
        return rc;
    hipStream_t s = (hipStream_t)stream;

    // host tables, built in a pinned staging slot
    Staging::Slot& slot = g_stage.slot[g_stage.next];
    g_stage.next = (g_stage.next + 1) % 4;
    if (slot.pending) {
        if (int rc = hip_status(hipEventSynchronize(slot.ev), "staging wait")) return rc;
        slot.pending = false;
    }
    if (!slot.ev) {
        if (int rc = hip_status(hipEventCreateWithFlags(&slot.ev, hipEventDisableTiming), "staging event")) return rc;
    }
    if (slot.size < (size_t)L.table_bytes) {
        if (slot.host) (void)hipHostFree(slot.host);
        slot.host = nullptr;
        slot.size = 0;
        const size_t want = (size_t)align_up(L.table_bytes, 1 << 16);
        if (int rc = hip_status(hipHostMalloc(&slot.host, want, hipHostMallocDefault), "staging alloc")) return rc;
        slot.size = want;
    }
    DetectRun R;
    fill_tables(frames, n_frames, n_models, tuning_of(params), L, static_cast<uint8_t*>(workspace),
                static_cast<uint8_t*>(workspace), static_cast<uint8_t*>(slot.host), R);

    int rc;
    StageMarks marks(g_prof.on);
    marks.mark(PD_STAGE_UPLOAD, s);
    if ((rc = hip_status(hipMemcpyAsync(workspace, slot.host, (size_t)L.table_bytes, hipMemcpyHostToDevice, s),
                         "table upload")))
        return rc;
    if ((rc = hip_status(hipEventRecord(slot.ev, s), "staging record"))) return rc;
    slot.pending = true;
    rc = enqueue_detect(R, L, tuning_of(params), weights, bias, n_models, params, thresholds, n_frames, boxes, cap,
                        counts, marks, s);
    marks.mark(PD_N_STAGES, s);
    marks.commit();
    return rc;
}

struct pd_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long long* stamps = nullptr;  // stage boundary clock stamps (captured with profiling on)
    void* tables = nullptr;                // the graph's own level, tile and NMS tables
};

int pd_graph_create(const pd_frame* frames, int n_frames, const float* weights, const float* bias, int n_models,
                    const pd_params* params, const double* thresholds, void* workspace, int64_t workspace_bytes,
                    pd_box* boxes, int cap, pd_counts* counts, void* stream, pd_graph** out) {
    if (!out) return fail(PD_E_ARG, "out is NULL");
    *out = nullptr;
    DetectLayout L;
    if (int rc = validate_detect(frames, n_frames, weights, bias, n_models, params, thresholds, workspace,
                                 workspace_bytes, boxes, cap, counts, L))
        return rc;
    // the tables are uploaded once, now, into memory the graph owns (so a
    // later pd_detect, capture or tuning run on the same workspace leaves
    // them alone); the graph holds only kernels
    std::vector<uint8_t> host((size_t)L.table_bytes);
    pd_graph* g = new pd_graph();
    hipStream_t s = (hipStream_t)stream;
    int rc = hip_status(hipMalloc(&g->tables, host.size()), "graph tables");
    if (rc) {
        delete g;
        return rc;
    }
    DetectRun R;
    fill_tables(frames, n_frames, n_models, tuning_of(params), L, static_cast<uint8_t*>(workspace),
                static_cast<uint8_t*>(g->tables), host.data(), R);
    rc = hip_status(hipMemcpyAsync(g->tables, host.data(), host.size(), hipMemcpyHostToDevice, s), "table upload");
    if (!rc) rc = hip_status(hipStreamSynchronize(s), "table upload");
    if (rc) {
        (void)hipFree(g->tables);
        delete g;
        return rc;
    }

    hipStream_t cs = nullptr;  // capture needs a stream other than the null stream
    if ((rc = hip_status(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream"))) {
        (void)hipFree(g->tables);
        delete g;
        return rc;
    }
    StageMarks marks(false);
    if (g_prof.on) {  // the graph's own stamp slots
        rc = hip_status(hipMalloc(&g->stamps, (PD_N_STAGES + 1) * sizeof(unsigned long long)), "stage stamps");
        marks.stamps = g->stamps;
    }
    if (!rc) rc = hip_status(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    if (!rc) {
        marks.mark(PD_STAGE_UPLOAD, cs);
        const int rc_enq = enqueue_detect(R, L, tuning_of(params), weights, bias, n_models, params, thresholds,
                                          n_frames, boxes, cap, counts, marks, cs);
        marks.mark(PD_N_STAGES, cs);
        const int rc_end = hip_status(hipStreamEndCapture(cs, &g->graph), "end capture");
        rc = rc_enq ? rc_enq : rc_end;
    }
    if (!rc) rc = hip_status(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0), "graph instantiate");
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        if (g->stamps) (void)hipFree(g->stamps);
        if (g->tables) (void)hipFree(g->tables);
        delete g;
        return rc;
    }
    *out = g;
    return PD_OK;
}

int pd_graph_launch(pd_graph* g, void* stream) {
    if (!g || !g->exec) return fail(PD_E_ARG, "graph is NULL");
    return hip_status(hipGraphLaunch(g->exec, (hipStream_t)stream), "graph launch");
}

int pd_graph_destroy(pd_graph* g) {
    if (!g) return PD_OK;
    int rc = PD_OK;
    if (g->exec) rc = hip_status(hipGraphExecDestroy(g->exec), "graph exec destroy");
    if (g->graph) {
        const int r2 = hip_status(hipGraphDestroy(g->graph), "graph destroy");
        rc = rc ? rc : r2;
    }
    if (g->stamps) {
        const int r3 = hip_status(hipFree(g->stamps), "stage stamps");
        rc = rc ? rc : r3;
    }
    if (g->tables) {
        const int r4 = hip_status(hipFree(g->tables), "graph tables");
        rc = rc ? rc : r4;
    }
    delete g;
    return rc;
}

int pd_graph_stage_ms(pd_graph* g, double* ms) {
    if (!g || !ms) return fail(PD_E_ARG, "graph or ms is NULL");
    if (!g->stamps) return fail(PD_E_ARG, "graph was captured without stage stamps");
    int dev = 0, khz = 0;
    int rc = hip_status(hipDeviceSynchronize(), "stage stamps");
    if (!rc) rc = hip_status(hipGetDevice(&dev), "stage stamps");
    if (!rc) rc = hip_status(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "clock rate");
    unsigned long long t[PD_N_STAGES + 1] = {};
    if (!rc) rc = hip_status(hipMemcpy(t, g->stamps, sizeof(t), hipMemcpyDeviceToHost), "stage stamps");
    if (rc) return rc;
    if (khz <= 0) return fail(PD_E_HIP, "device reports no constant clock rate");
    for (int k = 0; k < PD_N_STAGES; ++k) ms[k] = (double)(int64_t)(t[k + 1] - t[k]) / (double)khz;
    return PD_OK;
}

int pd_autotune(const pd_frame* frames, int n_frames, const float* weights, const float* bias, int n_models,
                const pd_params* params, const double* thresholds, void* workspace, int64_t workspace_bytes,
                pd_box* boxes, int cap, pd_counts* counts, int iters, pd_params* best, float* best_ms,
                void* stream) {
    if (!best) return fail(PD_E_ARG, "best is NULL");
    if (iters < 1 || iters > 1000) return fail(PD_E_ARG, "iters outside [1, 1000]");
    {
        DetectLayout L;
        if (int rc = validate_detect(frames, n_frames, weights, bias, n_models, params, thresholds, workspace,
                                     workspace_bytes, boxes, cap, counts, L))
            return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    const bool prof = g_prof.on;
    g_prof.on = false;  // tuning calls stay out of the stage profile
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = hip_status(hipEventCreate(&e0), "event");
    if (!rc) rc = hip_status(hipEventCreate(&e1), "event");
    // `iters` launches of a captured graph between two events: the device's
    // time alone (an eager call also builds and uploads its tables on the
    // host, which would favour shapes with fewer tiles, not faster kernels)
    auto time_run = [&](pd_graph* g, float* ms) -> int {
        int r = hip_status(hipEventRecord(e0, s), "event");
        for (int k = 0; k < iters && !r; ++k) r = pd_graph_launch(g, stream);
        if (!r) r = hip_status(hipEventRecord(e1, s), "event");
        if (!r) r = hip_status(hipEventSynchronize(e1), "event");
        if (!r) r = hip_status(hipEventElapsedTime(ms, e0, e1), "event");
        *ms /= (float)iters;
        return r;
    };
    // one round for one shape: capture (its tables go into the shared
    // workspace), one untimed launch, `iters` timed ones
    auto time_shape = [&](const pd_params& p, float* ms) -> int {
        pd_graph* g = nullptr;
        int r = pd_graph_create(frames, n_frames, weights, bias, n_models, &p, thresholds, workspace,
                                workspace_bytes, boxes, cap, counts, stream, &g);
        if (!r) r = pd_graph_launch(g, stream);
        if (!r) r = time_run(g, ms);
        if (g) {
            const int r2 = hip_status(hipStreamSynchronize(s), "tuning");
            const int r3 = pd_graph_destroy(g);
            r = r ? r : (r2 ? r2 : r3);
        }
        return r;
    };
    // a candidate against the current choice: three rounds timing both in
    // turn; each keeps its least time (clock and cache drift hits both alike,
    // and one timing alone is at its mercy)
    auto time_pair = [&](const pd_params& a, const pd_params& b, float* ms_a, float* ms_b) -> int {
        int r = PD_OK;
        for (int rep = 0; rep < 3 && !r; ++rep) {
            float ta = 0.0f, tb = 0.0f;
            r = time_shape(a, &ta);
            if (!r) r = time_shape(b, &tb);
            if (!r && (rep == 0 || ta < *ms_a)) *ms_a = ta;
            if (!r && (rep == 0 || tb < *ms_b)) *ms_b = tb;
        }
        return r;
    };
    pd_params cur = *params;
    const Tuning t0 = tuning_of(params);
    cur.tune_feat_rows = t0.feat_rows;
    cur.tune_score_rows = t0.score_rows;
    float cur_ms = 0.0f;
    // one knob at a time (the stages they shape are independent)
    const int feat_rows[] = {4, 6, 8, 10, 12, 14, 16};
    const int score_rows[] = {4, 8, 16};
    const int grids[] = {0, 256, 512, 1024, 2048};
    for (int knob = 0; knob < 3 && !rc; ++knob) {
        const int* vals = knob == 0 ? feat_rows : knob == 1 ? score_rows : grids;
        const int n = knob == 0 ? 7 : knob == 1 ? 3 : 5;
        if (knob == 1 && params->precision != PD_PREC_F32) continue;  // FP32 scoring only
        for (int v = 0; v < n && !rc; ++v) {
            pd_params c = cur;
            int& field = knob == 0 ? c.tune_feat_rows : knob == 1 ? c.tune_score_rows : c.tune_grid;
            const int now = knob == 0 ? cur.tune_feat_rows : knob == 1 ? cur.tune_score_rows : cur.tune_grid;
            if (vals[v] == now) continue;
            field = vals[v];
            float ms_cur = 0.0f, ms = 0.0f;
            rc = time_pair(cur, c, &ms_cur, &ms);
            if (!rc) cur_ms = ms_cur;
            if (!rc && ms < ms_cur) {
                cur = c;
                cur_ms = ms;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    g_prof.on = prof;
    if (rc) return rc;
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return PD_OK;
}

int pd_detect_candidates(const pd_frame* frames, int n_frames, const pd_params* params, int n_models,
                         const void* workspace, int64_t workspace_bytes, int frame, float* cand_score,
                         int32_t* cand_key, double* cand_s64, int cap, void* stream) {
    if (!check_params(params)) return PD_E_ARG;
    if (!frames || n_frames < 1 || frame < 0 || frame >= n_frames) return fail(PD_E_ARG, "bad frame index");
    if (!workspace || (cap > 0 && (!cand_score || !cand_key))) return fail(PD_E_ARG, "NULL pointer argument");
    DetectLayout L;
    if (!plan_detect(frames, n_frames, params, n_models, L)) return PD_E_SIZE;
    if (workspace_bytes < L.total) return fail(PD_E_WORKSPACE, "workspace smaller than pd_detect's");
    if (cand_s64 && !L.bf16) return fail(PD_E_ARG, "FP64 scores exist only with PD_PREC_BF16");
    if (cap < 0 || cap > L.cand_cap[frame])
        return fail(PD_E_SIZE, "cap outside [0, %d] (the frame's windows)", L.cand_cap[frame]);
    const uint8_t* ws = static_cast<const uint8_t*>(workspace);
    hipStream_t s = (hipStream_t)stream;
    const size_t o = (size_t)L.cand_off[frame];
    int rc;
    if ((rc = hip_status(hipMemcpyAsync(cand_score, ws + L.off_cscore + o * 4, (size_t)cap * 4,
                                        hipMemcpyDeviceToDevice, s),
                         "copy")))
        return rc;
    if ((rc = hip_status(hipMemcpyAsync(cand_key, ws + L.off_ckey + o * 16, (size_t)cap * 16,
                                        hipMemcpyDeviceToDevice, s),
                         "copy")))
        return rc;
    if (cand_s64)
        return hip_status(hipMemcpyAsync(cand_s64, ws + L.off_c64 + o * 8, (size_t)cap * 8, hipMemcpyDeviceToDevice, s),
                          "copy");
    return PD_OK;
}

int pd_nms(const float* cand_score, const int32_t* cand_key, int n, const int32_t* level_wh, int n_levels,
           pd_box* boxes, int cap, pd_counts* counts, void* stream) {
    if (n < 0 || n > PD_MAX_CANDIDATES) return fail(PD_E_SIZE, "n = %d outside [0, %d]", n, PD_MAX_CANDIDATES);
    if (n_levels < 1 || n_levels > PD_MAX_LEVELS) return fail(PD_E_SIZE, "n_levels outside [1, %d]", PD_MAX_LEVELS);
    if (!level_wh || !counts || (n > 0 && (!cand_score || !cand_key)) || (cap > 0 && !boxes) || cap < 0)
        return fail(PD_E_ARG, "NULL pointer argument");
    NmsGeom g{};
    g.n_levels = n_levels;
    for (int k = 0; k < n_levels; ++k) {
        g.wh[k][0] = level_wh[2 * k];
        g.wh[k][1] = level_wh[2 * k + 1];
        if (g.wh[k][0] < 1 || g.wh[k][1] < 1) return fail(PD_E_SIZE, "level %d has an empty size", k);
    }
    return hip_status(launch_nms_single(g, n, cand_score, reinterpret_cast<const int4*>(cand_key), boxes, cap,
                                        counts, (hipStream_t)stream),
                      "nms launch");
}

}  // extern "C"

// pd_detect on a workspace the caller names, with the tables' upload left to
// `upload` (given the host tables and the byte ranges of them in use, as
// (offset, size) pairs relative to the workspace start): for entry points
// that must not touch the staging ring's pinned memory.  No stage events.
#include "detect_workspace.h"

int pd::detect_on_workspace(const pd_frame* frames, int n_frames, const float* weights, const float* bias,
                            int n_models, const pd_params* params, const double* thresholds, void* workspace,
                            int64_t workspace_bytes, pd_box* boxes, int cap, pd_counts* counts, hipStream_t s,
                            TableUpload upload) {
    DetectLayout L;
    if (int rc = validate_detect(frames, n_frames, weights, bias, n_models, params, thresholds, workspace,
                                 workspace_bytes, boxes, cap, counts, L))
        return rc;
    std::vector<uint8_t> host((size_t)L.table_bytes);
    DetectRun R;
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    fill_tables(frames, n_frames, n_models, tuning_of(params), L, ws, ws, host.data(), R);
    // only the entries in use: the items, each tile list's used prefix (FP32
    // half-height score tiles follow the others), the NMS geometry and the
    // per-frame item index
    const int64_t tsz = (int64_t)sizeof(Tile), t0 = L.off_tiles;
    const int64_t ranges[7][2] = {
        {L.off_items, (int64_t)L.n_items * (int64_t)sizeof(LevelItem)},
        {t0, R.nrs * tsz},
        {t0 + L.n_rs * tsz, R.nft * tsz},
        {t0 + (L.n_rs + L.n_ft) * tsz, (int64_t)R.nsc * tsz},
        {t0 + (L.n_rs + L.n_ft + L.n_sc) * tsz, R.ncp * tsz},
        {t0 + (L.n_rs + L.n_ft + L.n_sc + L.n_cp) * tsz, R.npr * tsz},
        {L.off_geoms, L.table_bytes - L.off_geoms},
    };
    if (int rc = upload(host.data(), ws, &ranges[0][0], 7, s)) return rc;
    StageMarks marks(false);
    return enqueue_detect(R, L, tuning_of(params), weights, bias, n_models, params, thresholds, n_frames, boxes, cap,
                          counts, marks, s);
}
