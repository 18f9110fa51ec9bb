// Per-kernel-class event timing (see timer.hip).
#pragma once

#include <hip/hip_ext.h>

#include "sc_common.h"

namespace sc {

enum TimerClass {
    TC_WILSON_F32 = 0,    // one Wilson stencil pass, FP32, one column
    TC_WILSON_F64 = 1,    // one Wilson stencil pass, FP64, one column
    TC_GEMM_CN = 2,       // G = V^H W
    TC_GEMM_NN = 3,       // X += V Y
    TC_WILSON_F32_K = 4,  // one Wilson stencil pass, FP32, several columns
    TC_WILSON_F64_K = 5,  // one Wilson stencil pass, FP64, several columns
    TC_COUNT = 6
};

bool timer_on();

// Times the first kernel launched through SC_TLAUNCH while the scope is alive
// (on the scope's thread): that launch carries the scope's start and stop
// events in its own dispatch (hipExtLaunchKernel), so the recorded time is the
// kernel's and no marker packets enter the stream.  A scope whose launch does
// not go through SC_TLAUNCH records nothing.
class TimerScope {
   public:
    TimerScope(int cls, hipStream_t s, double bytes, double flops);
    ~TimerScope();
    // the armed scope of this thread, or nullptr
    static TimerScope* current();
    hipEvent_t start() const { return (hipEvent_t)a_; }
    hipEvent_t stop() const { return (hipEvent_t)b_; }
    void launched();  // the events are taken: later launches in the scope are not timed

   private:
    int cls_;
    hipStream_t s_;
    double bytes_, flops_;
    void* a_;
    void* b_;
    bool used_;
    TimerScope* prev_;
};

// hipLaunchKernelGGL, timed by the armed TimerScope if there is one
#define SC_TLAUNCH(KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                                                    \
    do {                                                                                                     \
        ::sc::TimerScope* sc_ts_ = ::sc::TimerScope::current();                                              \
        if (sc_ts_) {                                                                                        \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, sc_ts_->start(), sc_ts_->stop(), 0,   \
                                  __VA_ARGS__);                                                              \
            sc_ts_->launched();                                                                              \
        } else {                                                                                             \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                             \
        }                                                                                                    \
    } while (0)

// While a TimerMute is alive on a thread, no TimerScope of that thread times
// anything (no events are created or recorded).
class TimerMute {
   public:
    TimerMute();
    ~TimerMute();
};

sc_status timer_enable(int on);
sc_status timer_read(int cls, double* ms, int64_t* launches, double* bytes, double* flops);

}  // namespace sc
