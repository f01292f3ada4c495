// pd_detect_noalloc: pd_detect for callers that cannot allocate (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// Its workspace is `scratch`, a file-scope device array of
// PD_NOALLOC_SCRATCH_BYTES that the code-object loader allocates on every GPU
// the library runs on, held until the process ends.  In host code the
// array's name is only a stand-in: the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current,
// and only that address is used (kernel arguments).  The level and tile
// tables reach the device as kernel arguments (no staging buffer, no copy),
// so the call allocates no device or pinned host memory.  Every call on a GPU
// shares that GPU's array: overlapping calls on one GPU race.  The candidate
// and near counters are cleared by the first kernel of every call, and every
// other byte a call reads is written earlier in that call.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "detect_workspace.h"

namespace pd {
namespace {

static __device__ __align__(256) uint8_t scratch[PD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up on the first call on
// that device.
int scratch_base(void** out) {
    int dev = 0;
    if (int rc = hip_status(hipGetDevice(&dev), "current device")) return rc;
    if (dev < 0 || dev >= kMaxDevices) return fail(PD_E_HIP, "device index %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (int rc = hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address")) return rc;
        if (!p) return fail(PD_E_HIP, "the scratch array has no device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PD_OK;
}

// Up to kChunkWords words by value per launch, stored at `dst`.
constexpr int kChunkWords = 768;
struct TableChunk {
    uint32_t* dst;
    int32_t n_words;
    int32_t pad;
    uint32_t words[kChunkWords];
};

__global__ void table_chunk_kernel(TableChunk c) {
    for (int i = threadIdx.x; i < c.n_words; i += blockDim.x) c.dst[i] = c.words[i];
}

// The tables' ranges in use, carried to `dev` by table_chunk_kernel launches.
int upload_by_args(const uint8_t* host, uint8_t* dev, const int64_t* ranges, int n_ranges, hipStream_t s) {
    TableChunk c;
    c.pad = 0;
    for (int r = 0; r < n_ranges; ++r) {
        const int64_t off = ranges[2 * r], bytes = ranges[2 * r + 1];
        if ((off | bytes) & 3) return fail(PD_E_HIP, "table range %d not word aligned", r);
        for (int64_t o = off; o < off + bytes; o += 4 * kChunkWords) {
            const int64_t n = std::min<int64_t>(4 * kChunkWords, off + bytes - o);
            c.dst = reinterpret_cast<uint32_t*>(dev + o);
            c.n_words = (int32_t)(n / 4);
            std::memcpy(c.words, host + o, (size_t)n);
            table_chunk_kernel<<<1, 256, 0, s>>>(c);
            if (int rc = hip_status(hipGetLastError(), "table upload")) return rc;
        }
    }
    return PD_OK;
}

}  // namespace
}  // namespace pd

using namespace pd;

extern "C" int pd_detect_noalloc(const pd_frame* frames, int n_frames, const float* weights, const float* bias,
                                 int n_models, const pd_params* params, const double* thresholds, pd_box* boxes,
                                 int cap, pd_counts* counts, void* stream) {
    // the size check comes first, before any HIP call
    const int64_t need = pd_detect_workspace_bytes(frames, n_frames, params, n_models);
    if (need < 0) return (int)need;
    if (need > PD_NOALLOC_SCRATCH_BYTES)
        return fail(PD_E_WORKSPACE, "this batch needs %lld bytes of workspace, the static scratch holds %lld",
                    (long long)need, (long long)PD_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    if (int rc = scratch_base(&ws)) return rc;
    return detect_on_workspace(frames, n_frames, weights, bias, n_models, params, thresholds, ws,
                               PD_NOALLOC_SCRATCH_BYTES, boxes, cap, counts, (hipStream_t)stream, upload_by_args);
}
