// Per-kernel-class event timing (see timer.hip).
#pragma once

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

class TimerScope {
   public:
    TimerScope(int cls, hipStream_t s, double bytes, double flops);
    ~TimerScope();

   private:
    int cls_;
    hipStream_t s_;
    double bytes_, flops_;
    void* a_;
};

sc_status timer_enable(int on);
sc_status timer_read(int cls, double* ms, int64_t* launches, double* bytes, double* flops);

}  // namespace sc
