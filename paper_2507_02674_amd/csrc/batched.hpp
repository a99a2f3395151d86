// Context-owned state of the batched frame: side streams, events, captured
// graphs keyed by the argument bytes, and tuned tile sizes.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "glint.h"

namespace glint {

struct BatchedCache {
    static constexpr int kSideStreams = 4;  // environment branches (environment e on e % 4)
    static constexpr int kGroupStreams = 4; // shading branches (group g on g % 4)
    struct Entry {
        hipGraphExec_t exec = nullptr;
        void *workspace = nullptr; // the workspace its descriptors and tile tables live in
    };
    std::mutex mu;
    hipStream_t side[kSideStreams] = {};
    hipStream_t gside[kGroupStreams] = {};
    hipStream_t capture = nullptr; // graph capture (never the caller's stream)
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins; // one per environment: its products are ready
    std::vector<hipEvent_t> gdone; // one per shading group: its views are shaded
    std::map<std::string, Entry> graphs;
    std::map<long long, int> tuned; // (K, dtype, V, size class) -> pixels per workgroup
    int last_tile_px = 0;
    ~BatchedCache();
};

size_t batched_workspace_bytes(int n_views);
hipError_t frame_batched(BatchedCache &c, const glint_env_task *envs, int n_env, const glint_view *views,
                         int n_views, void *workspace, hipStream_t stream);

} // namespace glint
