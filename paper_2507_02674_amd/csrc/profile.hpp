// Optional per-kernel timing of the library's launches (for benchmarks).
//
// While a context's profiler is enabled, the entry points make it current
// for their thread (ProfScope) and every launch site (GLINT_LAUNCH) hands
// two HIP events to the dispatch itself (hipExtLaunchKernel), which
// timestamps the kernel's start and end without extra queue packets.
// Launches inside a stream capture are not timed.  With no current
// profiler GLINT_LAUNCH is a plain launch.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace glint {

struct ProfRecord {
    const char *name; // static string
    hipEvent_t start, stop;
};

struct ProfSummary {
    const char *name;
    double total_ms;
    int64_t launches;
};

struct Profiler {
    bool enabled = false;
    std::string only;                // comma-separated kernel names to time; empty: all
    bool selected(const char *name) const;
    std::vector<ProfRecord> records; // in launch order, not yet resolved
    std::vector<hipEvent_t> pool;    // events of resolved records, for reuse
    std::vector<ProfSummary> summary;
    ~Profiler();
    hipEvent_t event();
    // Creates events until the pool holds n (so that timed launches do not
    // create events themselves).
    void reserve(size_t n);
    // Waits for every recorded event, folds the records into `summary`
    // (adding to what it holds) and recycles the events.
    hipError_t collect();
    void reset();
};

Profiler *&current_profiler();

struct ProfScope {
    Profiler *prev;
    explicit ProfScope(Profiler *p) : prev(current_profiler()) { current_profiler() = (p && p->enabled) ? p : nullptr; }
    ~ProfScope() { current_profiler() = prev; }
};

class KernelTimer {
  public:
    KernelTimer(const char *name, hipStream_t s);
    ~KernelTimer();
    bool active() const { return p_ != nullptr; }
    hipEvent_t start() const { return start_; }
    hipEvent_t stop() const { return stop_; }

  private:
    Profiler *p_ = nullptr;
    const char *name_;
    hipEvent_t start_ = nullptr, stop_ = nullptr;
};

} // namespace glint

// Launches KERNEL (parenthesise template instances) like hipLaunchKernelGGL;
// timed under NAME while a profiler is current.
#define GLINT_LAUNCH(NAME, KERNEL, GRID, BLOCK, SHM, STREAM, ...)                                                \
    do {                                                                                                       \
        ::glint::KernelTimer glint_kt_(NAME, STREAM);                                                          \
        if (glint_kt_.active())                                                                                \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, glint_kt_.start(), glint_kt_.stop(), 0,   \
                                  __VA_ARGS__);                                                                \
        else                                                                                                   \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, __VA_ARGS__);                                 \
    } while (0)
