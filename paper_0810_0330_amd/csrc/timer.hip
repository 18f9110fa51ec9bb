// Optional per-kernel-class timing with HIP events, for benchmarks: when
// enabled, a sample of the launches of each stencil class (one in `every`,
// picked by a hash of the class's launch counter so that periodic launch
// patterns do not alias) and every contraction launch is bracketed by two
// events on the stream it runs on, and its algorithmic bytes and flops are
// recorded.  An event pair
// costs a few microseconds of queue time, so sampling keeps the timed run
// close to an untimed one.  Disabled (the default), the scopes cost one branch.
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
int g_every = 1;
uint64_t g_count[TC_COUNT];
std::vector<Rec> g_recs;      // recorded this session
std::vector<hipEvent_t> g_pool;  // reusable events
size_t g_pool_used = 0;

// splitmix64 finaliser of (class, launch counter); the contraction classes,
// whose launches last milliseconds, are always timed
bool sampled(int cls) {
    if (cls == TC_GEMM_CN || cls == TC_GEMM_NN) return true;
    uint64_t z = (g_count[cls]++) * 0x9E3779B97F4A7C15ull + (uint64_t)cls * 0xD1B54A32D192ED03ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return g_every <= 1 || z % (uint64_t)g_every == 0;
}

hipEvent_t take_event() {
    if (g_pool_used == g_pool.size()) {
        // timing only: no system-scope fence when the event is recorded, so
        // the timed dispatch does not end with a cache writeback and
        // invalidation that untimed launches do not pay (the stream is
        // synchronised before any elapsed time is read)
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        g_pool.push_back(e);
    }
    return g_pool[g_pool_used++];
}
}  // namespace

bool timer_on() { return g_on; }

namespace {
thread_local TimerScope* t_current = nullptr;
thread_local int t_mute = 0;
}

TimerMute::TimerMute() { ++t_mute; }
TimerMute::~TimerMute() { --t_mute; }

TimerScope* TimerScope::current() { return t_current; }

void TimerScope::launched() {
    used_ = true;
    t_current = prev_;
}

TimerScope::TimerScope(int cls, hipStream_t s, double bytes, double flops)
    : cls_(cls), s_(s), bytes_(bytes), flops_(flops), a_(nullptr), b_(nullptr), used_(false), prev_(t_current) {
    if (!g_on || t_mute > 0) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;  // not in graphs
    std::lock_guard<std::mutex> lk(g_mu);
    if (cls < 0 || cls >= TC_COUNT || !sampled(cls)) return;
    a_ = take_event();
    b_ = a_ ? take_event() : nullptr;
    if (!b_) {
        a_ = nullptr;
        return;
    }
    t_current = this;
}

TimerScope::~TimerScope() {
    if (!a_) return;
    if (t_current == this) t_current = prev_;
    if (!used_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.push_back({(hipEvent_t)a_, (hipEvent_t)b_, cls_, bytes_, flops_});
}

sc_status timer_enable(int every) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.clear();
    g_pool_used = 0;
    g_on = every > 0;
    g_every = every > 0 ? every : 1;
    for (auto& c : g_count) c = 0;
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
