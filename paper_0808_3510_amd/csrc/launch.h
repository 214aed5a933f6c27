// Host-side entry points of the kernel layer (kernels.hip), used by capi.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include "pat_internal.h"

namespace pat {

enum Op { OP_R = 0, OP_RT = 1, OP_A = 2, OP_AT = 3 };
enum Prec { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };

// Records a pair of events around every kernel launch when attached.
struct StageTimer {
  virtual void begin(const char* name, hipStream_t s) = 0;
  virtual void end(hipStream_t s) = 0;
  virtual ~StageTimer() {}
};

// Two extra streams and three events of one plan, for the batched launch:
// its radix classes run on their own streams, forked from the caller's
// stream and joined back into it.
struct ForkStreams {
  hipStream_t s[2] = {nullptr, nullptr};
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
};

// One operator over n instances.  hinst: host copies of the descriptors,
// dinst: their device addresses, hpoly: host copies of their tap-polynomial
// tables.  in/out: user arrays; ws: per-instance workspace bases.  counters:
// kNumCounters zeroed words of device memory for the persistent work queue,
// or nullptr for one workgroup per work item.
// fork: streams for the radix classes of a batch (nullptr, or with a timer
// attached: everything on `stream`).
hipError_t run_op(int prec, Op op, int n, const Inst* hinst, const Inst* const* dinst, const void* const* hpoly,
                  const void* const* in, void* const* out, void* const* ws, uint32_t* counters,
                  hipStream_t stream, StageTimer* timer, const ForkStreams* fork = nullptr);

// Stage a3 alone on user buffers (grid in, weighted node values out).
hipError_t run_interp(int prec, const Inst& hinst, const Inst* dinst, const void* hpoly, const void* grid,
                      void* out, hipStream_t stream, StageTimer* timer);

// Spreading alone (operator R^T's type-1 step) on user buffers: depth
// spectra in, oversampled grid lines out.
hipError_t run_spread(int prec, const Inst& hinst, const Inst* dinst, const void* hpoly, const void* vals,
                      void* grid, hipStream_t stream, StageTimer* timer);

// Error injection (the PAT_FAULT hook of the C ABI): the k-th kernel launch
// of the calling thread's next operator reports hipErrorLaunchFailure without
// launching anything (k = 0: none).  Set at the start of every call.
void set_launch_fault(int k);

// Device address of the current device's kScratchBytes scratch array (a
// file-scope __device__ array in kernels.hip), looked up with
// hipGetSymbolAddress on the first call per device and cached.
hipError_t scratch_buffer(void** ptr);

}  // namespace pat
