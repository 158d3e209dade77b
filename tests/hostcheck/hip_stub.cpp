// CPU stand-in for the HIP runtime calls and kernel launchers that the host
// library (host.cpp, server.cpp) makes, so that its host logic (validation,
// CSR/CSC building, row orders, chunk, panel and launch tables, batch and
// server bookkeeping) can run under AddressSanitizer and UBSan on a machine
// without a GPU.  "Device" memory is host memory; kernels do nothing except
// where the host reads a result back (the power iteration's estimates, the
// status words), which get fixed values.  Test infrastructure only.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "kernels.h"

namespace {
std::mutex g_mu;
std::map<char*, size_t> g_allocs;  // base -> size, for hipMemGetAddressRange
}  // namespace

extern "C" {
hipError_t hipMalloc(void** p, size_t n) {
  *p = std::malloc(n ? n : 1);
  if (!*p) return hipErrorOutOfMemory;
  std::lock_guard<std::mutex> lk(g_mu);
  g_allocs[(char*)*p] = n;
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_allocs.erase((char*)p);
  }
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { *p = std::malloc(n ? n : 1); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { if (n) std::memmove(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { if (n) std::memmove(d, s, n); return hipSuccess; }
hipError_t hipMemset(void* d, int v, size_t n) { std::memset(d, v, n); return hipSuccess; }
hipError_t hipMemGetAddressRange(hipDeviceptr_t* base, size_t* size, hipDeviceptr_t p) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_allocs.upper_bound((char*)p);
  if (it == g_allocs.begin()) return hipErrorInvalidValue;
  --it;
  if ((char*)p >= it->first + (it->second ? it->second : 1)) return hipErrorInvalidValue;
  *base = it->first;
  *size = it->second;
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) { *s = (hipStream_t)new char; return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete (char*)s; return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t)new char; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = (hipEvent_t)new char; return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete (char*)e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned int) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = (hipGraph_t)new char; return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  *e = (hipGraphExec_t)new char;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) { delete (char*)g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete (char*)e; return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 1.0f; return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  *v = a == hipDeviceAttributeWallClockRate ? 100000 : 256;
  return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_t* p, int) {
  std::memset(p, 0, sizeof *p);
  std::strcpy(p->gcnArchName, "stub");
  p->multiProcessorCount = 256;
  return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "stub"; }
int roctxRangePushA(const char*) { return 0; }
int roctxRangePop() { return 0; }
roctx_range_id_t roctxRangeStartA(const char*) { return 0; }
void roctxRangeStop(roctx_range_id_t) {}
void roctxMarkA(const char*) {}
}

namespace aapdhg {
hipError_t launch_loop_pass(const LaunchTables&, hipStream_t, int, hipEvent_t*) { return hipSuccess; }
hipError_t launch_loop(const LaunchTables&, hipStream_t, long long, unsigned int) { return hipSuccess; }
hipError_t launch_gram_refresh(const LaunchTables&, hipStream_t) { return hipSuccess; }
int gram_partials_per_tile(int mt) { return mt * (mt + 1) / 2 + mt; }
int loop_capacity(bool, int, bool) { return 512; }
int pass_capacity(bool, int, int pass, bool) { return pass == 0 ? 1024 : 768; }
hipError_t launch_start_point(const LPDesc&, bool, hipStream_t) { return hipSuccess; }
hipError_t launch_zero(void* p, size_t bytes, hipStream_t) { std::memset(p, 0, bytes); return hipSuccess; }
hipError_t static_scratch(void** out) {
  static unsigned char buf[STATIC_SCRATCH_BYTES];
  *out = buf;
  return hipSuccess;
}
hipError_t launch_scaling(const ScalingArgs&, hipStream_t) { return hipSuccess; }
hipError_t launch_unscale(const void*, const void*, const double*, bool, int, int, double*, double*, double*,
                          hipStream_t) { return hipSuccess; }
hipError_t launch_power_iteration(const LPDesc&, bool, int iters, unsigned long long, double*, double* est,
                                  hipStream_t) {
  for (int i = 0; i <= iters; ++i) est[i] = 1.0;  // ||K||^2 estimate of 1
  return hipSuccess;
}
hipError_t launch_gather_status(const LPDesc*, int count, int* out, hipStream_t) {
  for (int i = 0; i < count; ++i) out[i] = ST_ITER_LIMIT;  // every member stops after its first epoch
  return hipSuccess;
}
hipError_t launch_time_limit(const LPDesc*, int, hipStream_t) { return hipSuccess; }
hipError_t launch_to_f64(const void*, bool, double* dst, size_t len, hipStream_t) {
  std::memset(dst, 0, len * sizeof(double));
  return hipSuccess;
}
hipError_t launch_from_f64(const double*, void*, bool, size_t, hipStream_t) { return hipSuccess; }
}  // namespace aapdhg
