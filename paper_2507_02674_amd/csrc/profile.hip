// Per-kernel timing records (see profile.hpp).
#include <string.h>

#include "profile.hpp"

namespace glint {

Profiler *&current_profiler()
{
    thread_local Profiler *p = nullptr;
    return p;
}

Profiler::~Profiler() { reset(); }

bool Profiler::selected(const char *name) const
{
    if (only.empty()) return true;
    const size_t n = strlen(name);
    size_t pos = 0;
    while (pos <= only.size()) {
        size_t end = only.find(',', pos);
        if (end == std::string::npos) end = only.size();
        if (end - pos == n && only.compare(pos, n, name) == 0) return true;
        pos = end + 1;
    }
    return false;
}

hipEvent_t Profiler::event()
{
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void Profiler::reserve(size_t n)
{
    while (pool.size() < n) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return;
        pool.push_back(e);
    }
}

hipError_t Profiler::collect()
{
    hipError_t err = hipSuccess;
    for (const ProfRecord &r : records) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
        if (e != hipSuccess) {
            err = e;
        } else {
            ProfSummary *s = nullptr;
            for (ProfSummary &q : summary)
                if (strcmp(q.name, r.name) == 0) s = &q;
            if (!s) {
                summary.push_back({r.name, 0.0, 0});
                s = &summary.back();
            }
            s->total_ms += ms;
            s->launches += 1;
        }
        pool.push_back(r.start);
        pool.push_back(r.stop);
    }
    records.clear();
    return err;
}

void Profiler::reset()
{
    for (const ProfRecord &r : records) {
        (void)hipEventSynchronize(r.stop);
        pool.push_back(r.start);
        pool.push_back(r.stop);
    }
    records.clear();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
    summary.clear();
}

KernelTimer::KernelTimer(const char *name, hipStream_t s) : name_(name)
{
    Profiler *p = current_profiler();
    if (!p || !p->selected(name)) return;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone) return;
    start_ = p->event();
    stop_ = p->event();
    if (!start_ || !stop_) {
        if (start_) p->pool.push_back(start_);
        if (stop_) p->pool.push_back(stop_);
        start_ = stop_ = nullptr;
        return;
    }
    p_ = p;
}

KernelTimer::~KernelTimer()
{
    if (p_) p_->records.push_back({name_, start_, stop_});
}

} // namespace glint
