// Streaming video mode: frames arrive one at a time in host memory (Section
// 4.1 step 1 copies each to the GPU, step 5 brings the detections back), and
// the copies of one frame overlap the detection of its neighbours.
//
// A ring of `depth` slots; each owns a device frame, a pd_detect workspace,
// device and pinned-host result buffers, and the pd_detect kernel sequence
// captured once as a graph on its own buffers.  A push copies the frame into
// the slot's pinned buffer (host), then enqueues the upload on the upload
// stream, the graph on the compute stream (after the upload's event) and the
// download of counts and boxes on the download stream (after the graph's
// event).  Three streams at default priority, so the upload of frame n+1
// and the download of frame n-1 run while frame n is detected.  A pop waits
// for its slot's last event and hands the results to the caller; the slot is
// then free for a new push.
#include <cstring>
#include <vector>

#include "pd_internal.h"

using namespace pd;

struct pd_video {
    int w = 0, h = 0, pitch = 0, cap = 0, depth = 0;
    hipStream_t up = nullptr, compute = nullptr, down = nullptr;
    struct Slot {
        uint8_t* d_frame = nullptr;
        double* d_thr = nullptr;
        void* ws = nullptr;
        pd_box* d_boxes = nullptr;
        pd_counts* d_counts = nullptr;
        uint8_t* h_frame = nullptr;
        double* h_thr = nullptr;
        pd_box* h_boxes = nullptr;
        pd_counts* h_counts = nullptr;
        hipEvent_t ev_start = nullptr, ev_up = nullptr, ev_det = nullptr, ev_done = nullptr;
        pd_graph* graph = nullptr;
    };
    std::vector<Slot> slots;
    int head = 0, n_busy = 0;  // oldest pushed slot, slots pushed and not popped
};

namespace {

void release(pd_video* v) {
    for (auto s : {v->up, v->compute, v->down})
        if (s) (void)hipStreamSynchronize(s);
    for (pd_video::Slot& s : v->slots) {
        (void)pd_graph_destroy(s.graph);
        for (hipEvent_t e : {s.ev_start, s.ev_up, s.ev_det, s.ev_done})
            if (e) (void)hipEventDestroy(e);
        for (void* p : {(void*)s.d_frame, (void*)s.d_thr, s.ws, (void*)s.d_boxes, (void*)s.d_counts})
            if (p) (void)hipFree(p);
        for (void* p : {(void*)s.h_frame, (void*)s.h_thr, (void*)s.h_boxes, (void*)s.h_counts})
            if (p) (void)hipHostFree(p);
    }
    for (auto s : {v->up, v->compute, v->down})
        if (s) (void)hipStreamDestroy(s);
    delete v;
}

}  // namespace

extern "C" {

int pd_video_create(int w, int h, const pd_params* params, const float* weights, const float* bias, int n_models,
                    int cap, int depth, pd_video** out) {
    if (!out) return fail(PD_E_ARG, "out is NULL");
    *out = nullptr;
    if (depth < 1 || depth > PD_VIDEO_MAX_DEPTH) return fail(PD_E_SIZE, "depth %d outside [1, %d]", depth, PD_VIDEO_MAX_DEPTH);
    if (cap < 1) return fail(PD_E_SIZE, "cap %d < 1", cap);
    if (w < 1 || h < 1 || w > PD_MAX_DIM || h > PD_MAX_DIM) return fail(PD_E_SIZE, "frame %dx%d", w, h);
    if (!weights || !bias) return fail(PD_E_ARG, "NULL pointer argument");
    pd_frame desc{nullptr, w, h, (w + 15) / 16 * 16, 0};
    const int64_t ws_bytes = pd_detect_workspace_bytes(&desc, 1, params, n_models);
    if (ws_bytes < 0) return (int)ws_bytes;  // message set by the size query
    pd_video* v = new pd_video();
    v->w = w;
    v->h = h;
    v->pitch = desc.pitch;
    v->cap = cap;
    v->depth = depth;
    v->slots.resize(depth);
    int rc = PD_OK;
    for (hipStream_t* s : {&v->up, &v->compute, &v->down})
        if (!rc) rc = hip_status(hipStreamCreateWithFlags(s, hipStreamNonBlocking), "video stream");
    const size_t frame_bytes = (size_t)v->pitch * h;
    for (pd_video::Slot& s : v->slots) {
        if (rc) break;
        rc = hip_status(hipMalloc(&s.d_frame, frame_bytes), "video frame");
        if (!rc) rc = hip_status(hipMalloc(&s.d_thr, sizeof(double)), "video threshold");
        if (!rc) rc = hip_status(hipMalloc(&s.ws, (size_t)ws_bytes), "video workspace");
        if (!rc) rc = hip_status(hipMalloc(&s.d_boxes, sizeof(pd_box) * cap), "video boxes");
        if (!rc) rc = hip_status(hipMalloc(&s.d_counts, sizeof(pd_counts)), "video counts");
        if (!rc) rc = hip_status(hipHostMalloc(&s.h_frame, frame_bytes, hipHostMallocDefault), "video pinned frame");
        if (!rc) rc = hip_status(hipHostMalloc(&s.h_thr, sizeof(double), hipHostMallocDefault), "video pinned");
        if (!rc) rc = hip_status(hipHostMalloc(&s.h_boxes, sizeof(pd_box) * cap, hipHostMallocDefault), "video pinned");
        if (!rc) rc = hip_status(hipHostMalloc(&s.h_counts, sizeof(pd_counts), hipHostMallocDefault), "video pinned");
        if (!rc) rc = hip_status(hipEventCreate(&s.ev_start), "video event");
        if (!rc) rc = hip_status(hipEventCreate(&s.ev_done), "video event");
        if (!rc) rc = hip_status(hipEventCreateWithFlags(&s.ev_up, hipEventDisableTiming), "video event");
        if (!rc) rc = hip_status(hipEventCreateWithFlags(&s.ev_det, hipEventDisableTiming), "video event");
        if (!rc) {
            std::memset(s.h_frame, 0, frame_bytes);
            *s.h_thr = 0.0;
            rc = hip_status(hipMemcpyAsync(s.d_frame, s.h_frame, frame_bytes, hipMemcpyHostToDevice, v->compute),
                            "video frame clear");
        }
        if (!rc) {
            pd_frame f{s.d_frame, w, h, v->pitch, 0};
            rc = pd_graph_create(&f, 1, weights, bias, n_models, params, s.d_thr, s.ws, ws_bytes, s.d_boxes, cap,
                                 s.d_counts, v->compute, &s.graph);
        }
    }
    if (!rc) rc = hip_status(hipStreamSynchronize(v->compute), "video setup");
    if (rc) {
        release(v);
        return rc;
    }
    *out = v;
    return PD_OK;
}

int pd_video_push(pd_video* v, const uint8_t* frame, int pitch, double threshold) {
    if (!v || !frame) return fail(PD_E_ARG, "NULL pointer argument");
    if (pitch < v->w) return fail(PD_E_ARG, "pitch %d < width %d", pitch, v->w);
    if (v->n_busy == v->depth) return fail(PD_E_SIZE, "all %d slots hold frames not yet popped", v->depth);
    pd_video::Slot& s = v->slots[(v->head + v->n_busy) % v->depth];
    for (int y = 0; y < v->h; ++y) std::memcpy(s.h_frame + (size_t)y * v->pitch, frame + (size_t)y * pitch, v->w);
    *s.h_thr = threshold;
    int rc = hip_status(hipEventRecord(s.ev_start, v->up), "video record");
    if (!rc)
        rc = hip_status(hipMemcpyAsync(s.d_frame, s.h_frame, (size_t)v->pitch * v->h, hipMemcpyHostToDevice, v->up),
                        "video upload");
    if (!rc) rc = hip_status(hipMemcpyAsync(s.d_thr, s.h_thr, sizeof(double), hipMemcpyHostToDevice, v->up), "video upload");
    if (!rc) rc = hip_status(hipEventRecord(s.ev_up, v->up), "video record");
    if (!rc) rc = hip_status(hipStreamWaitEvent(v->compute, s.ev_up, 0), "video wait");
    if (!rc) rc = pd_graph_launch(s.graph, v->compute);
    if (!rc) rc = hip_status(hipEventRecord(s.ev_det, v->compute), "video record");
    if (!rc) rc = hip_status(hipStreamWaitEvent(v->down, s.ev_det, 0), "video wait");
    if (!rc)
        rc = hip_status(hipMemcpyAsync(s.h_counts, s.d_counts, sizeof(pd_counts), hipMemcpyDeviceToHost, v->down),
                        "video download");
    if (!rc)
        rc = hip_status(hipMemcpyAsync(s.h_boxes, s.d_boxes, sizeof(pd_box) * v->cap, hipMemcpyDeviceToHost, v->down),
                        "video download");
    if (!rc) rc = hip_status(hipEventRecord(s.ev_done, v->down), "video record");
    if (rc) return rc;  // the slot stays free; streams hold whatever was enqueued
    ++v->n_busy;
    return PD_OK;
}

int pd_video_pop(pd_video* v, pd_box* boxes, int cap, pd_counts* counts, float* device_ms) {
    if (!v || !counts || (!boxes && cap > 0)) return fail(PD_E_ARG, "NULL pointer argument");
    if (v->n_busy == 0) return fail(PD_E_ARG, "no frame pushed and not yet popped");
    pd_video::Slot& s = v->slots[v->head];
    if (int rc = hip_status(hipEventSynchronize(s.ev_done), "video wait")) return rc;
    if (device_ms)
        if (int rc = hip_status(hipEventElapsedTime(device_ms, s.ev_start, s.ev_done), "video timing")) return rc;
    *counts = *s.h_counts;
    const int n = std::min(std::min(s.h_counts->kept, v->cap), std::max(cap, 0));
    if (n > 0) std::memcpy(boxes, s.h_boxes, sizeof(pd_box) * n);
    v->head = (v->head + 1) % v->depth;
    --v->n_busy;
    if (s.h_counts->overflow || s.h_counts->kept > cap)
        return fail(PD_E_OVERFLOW, "frame results truncated: %d candidates, %d kept, %d boxes room",
                    s.h_counts->candidates, s.h_counts->kept, cap);
    return PD_OK;
}

int pd_video_destroy(pd_video* v) {
    if (v) release(v);
    return PD_OK;
}

}  // extern "C"
