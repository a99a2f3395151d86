// Batched frame: many environments and views in one HIP graph launch.
//
// Set-up (first call per argument set): validate, upload per-view shading
// descriptors and per-group tile tables into the caller's workspace, time
// the shading launch for each candidate tile size, then capture the frame:
// one branch per environment on the context's side streams (partition ->
// source chain -> prefilter) and one branch per (K, vertices, form) shading
// group on the group streams, each group waiting only for the environments
// its views are lit by, all joined on the capture stream.  Replays: one
// hipGraphLaunch.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "batched.hpp"
#include "device.hpp"
#include "internal.hpp"

namespace glint {

namespace {

constexpr int kTileCandidates[] = {64, 128, 256}; // pixels per block (multiples of one wave, <= 256)

struct Group {
    int K, V;
    bool surrogate;           // views shaded with their environment's network
    std::vector<int> views;   // indices into the caller's view array
    int64_t tiles = 0;
    size_t desc_off = 0, tile_off = 0; // byte offsets in the workspace
    int tile_px = 256;
};

int64_t size_class(int64_t pixels)
{
    int64_t c = 0;
    while ((int64_t(1) << (c + 1)) <= pixels) ++c;
    return c;
}

// Uploads descriptors + tile tables for tile size px; returns a HIP error.
hipError_t upload_group(const Group &g, const glint_env_task *envs, const glint_view *views, int px,
                        void *workspace, hipStream_t stream)
{
    const size_t ab = shade_args_bytes();
    std::vector<unsigned char> desc(ab * g.views.size());
    std::vector<int64_t> tile0(g.views.size());
    int64_t t = 0;
    for (size_t q = 0; q < g.views.size(); ++q) {
        const glint_view &v = views[g.views[q]];
        const glint_env_task &e = envs[v.env_index];
        glint_env env{e.ind_pyr, e.rgb_pyr, e.levels, e.lut_S, e.lut_E, e.R, e.partition.K, e.prefilter.num_mips,
                      e.prefilter.dtype, e.quantile_tail};
        make_shade_args(desc.data() + q * ab, v.gbuf, v.num_pixels, env, v.shade, v.radiance,
                        g.surrogate ? v.surrogate_F : nullptr);
        tile0[q] = t;
        t += (v.num_pixels + px - 1) / px;
    }
    char *ws = static_cast<char *>(workspace);
    hipError_t err = hipMemcpyAsync(ws + g.desc_off, desc.data(), desc.size(), hipMemcpyHostToDevice, stream);
    if (err != hipSuccess) return err;
    err = hipMemcpyAsync(ws + g.tile_off, tile0.data(), tile0.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                         stream);
    if (err != hipSuccess) return err;
    return hipStreamSynchronize(stream); // host staging buffers go out of scope
}

int64_t group_tiles(const Group &g, const glint_view *views, int px)
{
    int64_t t = 0;
    for (int vi : g.views) t += (views[vi].num_pixels + px - 1) / px;
    return t;
}

hipError_t launch_env(const glint_env_task &e, hipStream_t s)
{
    hipError_t err = launch_partition(e.env, e.R, e.partition.K, e.partition.ell, e.partition.level_mode,
                                      e.partition.weight_space, e.partition_workspace, e.levels, e.ind_j, e.ind_t, s);
    if (err != hipSuccess) return err;
    return launch_prefilter(e.env, e.ind_j, e.ind_t, e.R, e.partition.K, e.prefilter.num_mips, e.prefilter.taps,
                            (int)e.prefilter.dtype, e.prefilter_workspace, e.ind_pyr, e.rgb_pyr, s);
}

// Network lookups of a surrogate group's views (one launch per view).
hipError_t launch_lookups(const Group &g, const glint_env_task *envs, const glint_view *views, hipStream_t s)
{
    if (!g.surrogate) return hipSuccess;
    for (int vi : g.views) {
        const glint_view &v = views[vi];
        const glint_env_task &e = envs[v.env_index];
        hipError_t err = launch_mlp_lookup(v.gbuf, v.num_pixels, e.partition.K, e.surrogate_w, e.surrogate_w_bf16,
                                           v.surrogate_F, s);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_group(const Group &g, int dtype, void *workspace, hipStream_t s)
{
    char *ws = static_cast<char *>(workspace);
    return launch_shade_views(g.K, dtype, g.V, g.surrogate, ws + g.desc_off,
                              reinterpret_cast<const int64_t *>(ws + g.tile_off), (int)g.views.size(), g.tiles,
                              g.tile_px, s);
}

} // namespace

size_t batched_workspace_bytes(int n_views)
{
    // descriptors and tile tables of at most n_views views, each group
    // aligned to 256 bytes (at most 16 groups: K in {2,4,8,16} x V in {1,6}
    // x plain/surrogate)
    return (size_t)n_views * (shade_args_bytes() + sizeof(int64_t)) + 32 * 256;
}

BatchedCache::~BatchedCache()
{
    for (auto &kv : graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    }
    for (int i = 0; i < kSideStreams; ++i) {
        if (side[i]) (void)hipStreamDestroy(side[i]);
    }
    for (int i = 0; i < kGroupStreams; ++i) {
        if (gside[i]) (void)hipStreamDestroy(gside[i]);
    }
    if (capture) (void)hipStreamDestroy(capture);
    if (fork) (void)hipEventDestroy(fork);
    for (auto &ev : joins) (void)hipEventDestroy(ev);
    for (auto &ev : gdone) (void)hipEventDestroy(ev);
}

// Streams once per context; events grow to n_env environment joins and
// n_groups group completions (the capture indexes each vector only below
// its size, checked there).
static hipError_t ensure_streams(BatchedCache &c, int n_env, int n_groups)
{
    if (!c.side[0]) {
        for (int i = 0; i < BatchedCache::kSideStreams; ++i) {
            hipError_t err = hipStreamCreateWithFlags(&c.side[i], hipStreamNonBlocking);
            if (err != hipSuccess) return err;
        }
        for (int i = 0; i < BatchedCache::kGroupStreams; ++i) {
            hipError_t err = hipStreamCreateWithFlags(&c.gside[i], hipStreamNonBlocking);
            if (err != hipSuccess) return err;
        }
        hipError_t e2 = hipStreamCreateWithFlags(&c.capture, hipStreamNonBlocking);
        if (e2 != hipSuccess) return e2;
        hipError_t err = hipEventCreateWithFlags(&c.fork, hipEventDisableTiming);
        if (err != hipSuccess) return err;
    }
    while ((int)c.joins.size() < n_env) {
        hipEvent_t ev;
        hipError_t err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (err != hipSuccess) return err;
        c.joins.push_back(ev);
    }
    while ((int)c.gdone.size() < n_groups) {
        hipEvent_t ev;
        hipError_t err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (err != hipSuccess) return err;
        c.gdone.push_back(ev);
    }
    return hipSuccess;
}

hipError_t frame_batched(BatchedCache &c, const glint_env_task *envs, int n_env, const glint_view *views,
                         int n_views, void *workspace, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(c.mu);
    std::string key;
    key.append(reinterpret_cast<const char *>(envs), sizeof(glint_env_task) * n_env);
    key.append(reinterpret_cast<const char *>(views), sizeof(glint_view) * n_views);
    key.append(reinterpret_cast<const char *>(&workspace), sizeof(workspace));
    auto it = c.graphs.find(key);
    if (it != c.graphs.end()) return hipGraphLaunch(it->second.exec, stream);

    hipError_t err;
    const int dtype = (int)envs[0].prefilter.dtype;

    // A graph reads its descriptors and tile tables from the workspace, where
    // this set-up call writes its own: a workspace holds one argument set, so
    // every graph captured on it is dropped (it would read the new set with
    // its old grid sizes).  Earlier launches of those graphs on `stream` are
    // ordered before the uploads below; the wait lets them finish first.
    if ((err = hipStreamSynchronize(stream)) != hipSuccess) return err;
    for (auto g = c.graphs.begin(); g != c.graphs.end();) {
        if (g->second.workspace == workspace) {
            (void)hipGraphExecDestroy(g->second.exec);
            g = c.graphs.erase(g);
        } else {
            ++g;
        }
    }

    // groups by (K, V, form), views in caller order
    std::vector<Group> groups;
    for (int v = 0; v < n_views; ++v) {
        const glint_env_task &e = envs[views[v].env_index];
        const int K = e.partition.K, V = views[v].shade.vertices;
        const bool S = e.surrogate_w != nullptr;
        auto g = std::find_if(groups.begin(), groups.end(),
                              [&](const Group &x) { return x.K == K && x.V == V && x.surrogate == S; });
        if (g == groups.end()) {
            groups.push_back(Group{K, V, S, {}, 0, 0, 0, 256});
            g = groups.end() - 1;
        }
        g->views.push_back(v);
    }
    if ((err = ensure_streams(c, n_env, (int)groups.size())) != hipSuccess) return err;
    size_t off = 0;
    for (auto &g : groups) {
        g.desc_off = off;
        off += (shade_args_bytes() * g.views.size() + 255) / 256 * 256;
        g.tile_off = off;
        off += (sizeof(int64_t) * g.views.size() + 255) / 256 * 256;
    }

    // environment products once, eagerly, so the tuning runs shade real data
    for (int e = 0; e < n_env; ++e) {
        if ((err = launch_env(envs[e], stream)) != hipSuccess) return err;
    }
    // autotune the tile size per group (cached per K, dtype, V, size class)
    // the timing events live until this scope ends, on every return path
    struct TimingEvents {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~TimingEvents()
        {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } tev;
    if ((err = hipEventCreate(&tev.e[0])) != hipSuccess) return err;
    if ((err = hipEventCreate(&tev.e[1])) != hipSuccess) return err;
    hipEvent_t t0 = tev.e[0], t1 = tev.e[1];
    int64_t biggest = -1;
    for (auto &g : groups) {
        int64_t px_total = 0;
        for (int vi : g.views) px_total += views[vi].num_pixels;
        const long long tkey = ((long long)g.K << 40) | ((long long)dtype << 32) | ((long long)g.surrogate << 24) |
                               ((long long)g.V << 16) | size_class(px_total);
        auto tuned = c.tuned.find(tkey);
        if (tuned != c.tuned.end()) {
            g.tile_px = tuned->second;
        } else {
            float best = 1e30f;
            if ((err = launch_lookups(g, envs, views, stream)) != hipSuccess) return err;
            for (int px : kTileCandidates) {
                g.tile_px = px;
                g.tiles = group_tiles(g, views, px);
                if ((err = upload_group(g, envs, views, px, workspace, stream)) != hipSuccess) return err;
                float ms_sum = 0.0f;
                for (int rep = 0; rep < 3; ++rep) {
                    if ((err = hipEventRecord(t0, stream)) != hipSuccess) return err;
                    if ((err = launch_group(g, dtype, workspace, stream)) != hipSuccess) return err;
                    if ((err = hipEventRecord(t1, stream)) != hipSuccess) return err;
                    if ((err = hipEventSynchronize(t1)) != hipSuccess) return err;
                    float ms = 0.0f;
                    if ((err = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) return err;
                    if (rep > 0) ms_sum += ms; // first repetition warms caches
                }
                if (ms_sum < best) {
                    best = ms_sum;
                    c.tuned[tkey] = px;
                }
            }
            g.tile_px = c.tuned[tkey];
        }
        g.tiles = group_tiles(g, views, g.tile_px);
        if ((err = upload_group(g, envs, views, g.tile_px, workspace, stream)) != hipSuccess) return err;
        if (px_total > biggest) {
            biggest = px_total;
            c.last_tile_px = g.tile_px;
        }
    }

    // capture on the context's own stream (the caller's may be the legacy
    // NULL stream, which cannot be captured): a branch per environment, a
    // branch per shading group after the environments it reads, all joined
    // on the capture stream.  The graph is then launched on the caller's
    // stream.
    if ((int)c.joins.size() < n_env || (int)c.gdone.size() < (int)groups.size()) return hipErrorInvalidValue;
    hipGraph_t graph = nullptr;
    hipStream_t cs = c.capture;
    if ((err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) return err;
    hipError_t cap = hipEventRecord(c.fork, cs);
    for (int e = 0; e < n_env && cap == hipSuccess; ++e) {
        hipStream_t s = c.side[e % BatchedCache::kSideStreams];
        cap = hipStreamWaitEvent(s, c.fork, 0);
        if (cap == hipSuccess) cap = launch_env(envs[e], s);
        if (cap == hipSuccess) cap = hipEventRecord(c.joins[e], s);
    }
    for (size_t gi = 0; gi < groups.size() && cap == hipSuccess; ++gi) {
        const Group &g = groups[gi];
        hipStream_t s = c.gside[gi % BatchedCache::kGroupStreams];
        std::vector<char> needs(n_env, 0);
        for (int vi : g.views) {
            const int e = views[vi].env_index;
            if (e < 0 || e >= n_env) { cap = hipErrorInvalidValue; break; }
            needs[e] = 1;
        }
        if (cap == hipSuccess) cap = hipStreamWaitEvent(s, c.fork, 0);
        for (int e = 0; e < n_env && cap == hipSuccess; ++e)
            if (needs[e]) cap = hipStreamWaitEvent(s, c.joins[e], 0);
        if (cap == hipSuccess) cap = launch_lookups(g, envs, views, s);
        if (cap == hipSuccess) cap = launch_group(g, dtype, workspace, s);
        if (cap == hipSuccess) cap = hipEventRecord(c.gdone[gi], s);
    }
    // every branch rejoins the capture stream (environments no view reads too)
    for (int e = 0; e < n_env && cap == hipSuccess; ++e) cap = hipStreamWaitEvent(cs, c.joins[e], 0);
    for (size_t gi = 0; gi < groups.size() && cap == hipSuccess; ++gi) cap = hipStreamWaitEvent(cs, c.gdone[gi], 0);
    err = hipStreamEndCapture(cs, &graph);
    if (cap != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return cap;
    }
    if (err != hipSuccess) return err;
    hipGraphExec_t exec = nullptr;
    err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (err != hipSuccess) return err;
    if (c.graphs.size() >= 16) { // bounded cache: drop one entry
        (void)hipGraphExecDestroy(c.graphs.begin()->second.exec);
        c.graphs.erase(c.graphs.begin());
    }
    c.graphs[key] = BatchedCache::Entry{exec, workspace};
    return hipGraphLaunch(exec, stream);
}

} // namespace glint
