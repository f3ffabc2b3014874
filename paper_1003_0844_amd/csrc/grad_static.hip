// fstat_grad_static: F and its gradient at candidate parameters, like
// fstat_grad, without any device allocation.  The forward state that
// fstat_grad keeps in the plan's workspace (grown with hipMalloc on demand)
// lives here in a fixed device array, so the call suits callers that cannot
// allocate: code under HIP graph capture, serving loops.
//
// Each GPU holds its own copy of the array; its address is taken once per
// device with hipGetSymbolAddress on the first call on that device (with the
// device current) and reused.  Host code never passes the array's name to a
// kernel: in host code it is only a stand-in for the symbol.
#include <mutex>

#include "../../include/fstat.h"
#include "internal.h"

// the plan's device segment table (defined in api.hip)
const SegDev* fstat_plan_device_segments(fstat_plan_t p, int* nseg, int* device);

namespace {

// room for FSTAT_GRAD_STATIC_MAX candidates of FSTATE doubles: 4 MiB per GPU
static __device__ __align__(256) double scratch[FSTAT_GRAD_STATIC_MAX * FSTATE];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

// The array's address on the current device (taken once per device).
hipError_t scratch_on(int dev, double** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" fstat_status fstat_grad_static(fstat_plan_t p, const double* params, const int32_t* seg, int64_t n,
                                          double* F, double* dF, void* hip_stream) {
  if (!p || !params || n <= 0 || !F || !dF) return FSTAT_EINVAL;
  if (n > FSTAT_GRAD_STATIC_MAX) return FSTAT_EUNSUPPORTED;
  int nseg = 0, device = 0;
  const SegDev* d_segs = fstat_plan_device_segments(p, &nseg, &device);
  if (!d_segs) return FSTAT_EINVAL;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return FSTAT_EDEVICE;
  double* state = nullptr;
  hipError_t e = scratch_on(device, &state);
  const hipStream_t st = (hipStream_t)hip_stream;
  // every candidate's state is written by the forward kernel before the
  // adjoint reads it: nothing needs clearing
  if (e == hipSuccess) e = fsk::grad_forward(d_segs, nseg, seg, params, n, F, state, st);
  if (e == hipSuccess) e = fsk::grad_adjoint(d_segs, nseg, seg, params, n, state, nullptr, dF, st);
  (void)hipSetDevice(prev);
  if (e == hipSuccess) return FSTAT_OK;
  return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? FSTAT_ENOMEM : FSTAT_EDEVICE;
}
