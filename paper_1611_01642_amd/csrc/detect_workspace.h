// pd_detect on a workspace and table upload chosen by the caller (internal).
#pragma once

#include "pd_internal.h"

namespace pd {

// Uploads the host tables `host` to `dev`: n_ranges (offset, size) byte
// ranges relative to both, every offset and size a multiple of 4.
using TableUpload = int (*)(const uint8_t* host, uint8_t* dev, const int64_t* ranges, int n_ranges, hipStream_t s);

// pd_detect's checks, tables and kernel sequence on `workspace`, the tables'
// entries in use carried by `upload`; no stage events.
int detect_on_workspace(const pd_frame* frames, int n_frames, const float* weights, const float* bias,
                        int n_models, const pd_params* params, const double* thresholds, void* workspace,
                        int64_t workspace_bytes, pd_box* boxes, int cap, pd_counts* counts, hipStream_t s,
                        TableUpload upload);

}  // namespace pd
