// Training checkpoints of the learned window pruner: the network's
// parameters, Adam's two moment vectors, the number of Adam steps taken and
// the seed of the training order, so that an interrupted training run
// resumes exactly where it stopped.
//
// File layout (little endian):
//   bytes 0..7    magic "PDPRUNE1"
//   u32           format version (1)
//   u32           n = PD_PRUNER_PARAMS
//   i64           step
//   u64           seed
//   f32 x n       parameters, then f32 x n first moments, f32 x n second moments
//   u64           FNV-1a 64 of every byte before it
// The device vectors are copied through host memory with plain HIP copies on
// the caller's stream, which is synchronised before the call returns.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pd_internal.h"

using namespace pd;

namespace {

constexpr char kMagic[8] = {'P', 'D', 'P', 'R', 'U', 'N', 'E', '1'};
constexpr uint32_t kVersion = 1;
constexpr size_t kHeader = 8 + 4 + 4 + 8 + 8;

uint64_t fnv1a64(const uint8_t* p, size_t n) {
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

template <typename T>
void put(std::vector<uint8_t>& b, size_t at, T v) {
    std::memcpy(b.data() + at, &v, sizeof(T));
}

template <typename T>
T get(const std::vector<uint8_t>& b, size_t at) {
    T v;
    std::memcpy(&v, b.data() + at, sizeof(T));
    return v;
}

}  // namespace

extern "C" {

int pd_pruner_save(const char* path, const float* params, const float* adam_m, const float* adam_v, int64_t step,
                   uint64_t seed, void* stream) {
    if (!path || !params || !adam_m || !adam_v) return fail(PD_E_ARG, "NULL pointer argument");
    if (step < 0) return fail(PD_E_ARG, "step must be >= 0");
    constexpr size_t n = PD_PRUNER_PARAMS, vec = n * sizeof(float);
    std::vector<uint8_t> buf(kHeader + 3 * vec + 8);
    std::memcpy(buf.data(), kMagic, 8);
    put<uint32_t>(buf, 8, kVersion);
    put<uint32_t>(buf, 12, (uint32_t)n);
    put<int64_t>(buf, 16, step);
    put<uint64_t>(buf, 24, seed);
    hipStream_t s = (hipStream_t)stream;
    const float* src[3] = {params, adam_m, adam_v};
    for (int k = 0; k < 3; ++k)
        if (int rc = hip_status(hipMemcpyAsync(buf.data() + kHeader + k * vec, src[k], vec, hipMemcpyDeviceToHost, s),
                                "checkpoint copy"))
            return rc;
    if (int rc = hip_status(hipStreamSynchronize(s), "checkpoint copy")) return rc;
    put<uint64_t>(buf, kHeader + 3 * vec, fnv1a64(buf.data(), kHeader + 3 * vec));
    // write a sibling file, then rename it over the target: a reader never sees
    // a half-written checkpoint
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(PD_E_IO, "cannot open %s for writing", tmp.c_str());
    const bool ok = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
    const bool closed = std::fclose(f) == 0;
    if (!ok || !closed) {
        std::remove(tmp.c_str());
        return fail(PD_E_IO, "cannot write %s", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(PD_E_IO, "cannot rename %s to %s", tmp.c_str(), path);
    }
    return PD_OK;
}

int pd_pruner_load(const char* path, float* params, float* adam_m, float* adam_v, int64_t* step, uint64_t* seed,
                   void* stream) {
    if (!path || !params || !step || !seed) return fail(PD_E_ARG, "NULL pointer argument");
    constexpr size_t n = PD_PRUNER_PARAMS, vec = n * sizeof(float);
    std::vector<uint8_t> buf(kHeader + 3 * vec + 8);
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(PD_E_IO, "cannot open %s", path);
    const size_t got = std::fread(buf.data(), 1, buf.size(), f);
    const bool longer = std::fgetc(f) != EOF;
    std::fclose(f);
    if (got != buf.size() || longer) return fail(PD_E_IO, "%s: not a pruner checkpoint (size)", path);
    if (std::memcmp(buf.data(), kMagic, 8) != 0) return fail(PD_E_IO, "%s: not a pruner checkpoint (magic)", path);
    if (get<uint32_t>(buf, 8) != kVersion || get<uint32_t>(buf, 12) != (uint32_t)n)
        return fail(PD_E_IO, "%s: unsupported version or parameter count", path);
    if (get<uint64_t>(buf, kHeader + 3 * vec) != fnv1a64(buf.data(), kHeader + 3 * vec))
        return fail(PD_E_IO, "%s: checksum mismatch", path);
    const int64_t st = get<int64_t>(buf, 16);
    if (st < 0) return fail(PD_E_IO, "%s: negative step", path);
    hipStream_t s = (hipStream_t)stream;
    float* dst[3] = {params, adam_m, adam_v};
    for (int k = 0; k < 3; ++k) {
        if (!dst[k]) continue;  // a caller resuming inference only may skip the moments
        if (int rc = hip_status(hipMemcpyAsync(dst[k], buf.data() + kHeader + k * vec, vec, hipMemcpyHostToDevice, s),
                                "checkpoint copy"))
            return rc;
    }
    if (int rc = hip_status(hipStreamSynchronize(s), "checkpoint copy")) return rc;
    *step = st;
    *seed = get<uint64_t>(buf, 24);
    return PD_OK;
}

}  // extern "C"
