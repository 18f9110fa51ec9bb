// Optional per-kernel-class timing with HIP events, for benchmarks: when
// enabled, every launch of an instrumented kernel is bracketed by two events
// on the stream it runs on, and its algorithmic bytes and flops are recorded.
// Disabled (the default), the scopes cost one branch.
#include <mutex>
#include <vector>

#include "sc_timer.h"

namespace sc {

namespace {
struct Rec {
    hipEvent_t a, b;
    int cls;
    double bytes, flops;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;      // recorded this session
std::vector<hipEvent_t> g_pool;  // reusable events
size_t g_pool_used = 0;

hipEvent_t take_event() {
    if (g_pool_used == g_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_pool.push_back(e);
    }
    return g_pool[g_pool_used++];
}
}  // namespace

bool timer_on() { return g_on; }

TimerScope::TimerScope(int cls, hipStream_t s, double bytes, double flops)
    : cls_(cls), s_(s), bytes_(bytes), flops_(flops), a_(nullptr) {
    if (!g_on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;  // not in graphs
    std::lock_guard<std::mutex> lk(g_mu);
    a_ = take_event();
    if (a_) hipEventRecord((hipEvent_t)a_, s_);
}

TimerScope::~TimerScope() {
    if (!a_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b = take_event();
    if (!b) return;
    hipEventRecord(b, s_);
    g_recs.push_back({(hipEvent_t)a_, b, cls_, bytes_, flops_});
}

sc_status timer_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.clear();
    g_pool_used = 0;
    g_on = on != 0;
    return SC_OK;
}

sc_status timer_read(int cls, double* ms, int64_t* launches, double* bytes, double* flops) {
    std::lock_guard<std::mutex> lk(g_mu);
    double t = 0.0, by = 0.0, fl = 0.0;
    int64_t nl = 0;
    for (const Rec& r : g_recs) {
        if (r.cls != cls) continue;
        SC_HIP(hipEventSynchronize(r.b));
        float e = 0.0f;
        SC_HIP(hipEventElapsedTime(&e, r.a, r.b));
        t += e;
        by += r.bytes;
        fl += r.flops;
        ++nl;
    }
    *ms = t;
    *launches = nl;
    *bytes = by;
    *flops = fl;
    return SC_OK;
}

}  // namespace sc
