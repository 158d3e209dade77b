// Serving loop of the AA-PDHG library (continuous batching of LP requests).
#include "runtime.h"

using namespace aapdhg;

extern "C" {

aapdhg_status aapdhg_server_start(size_t, int32_t, const aapdhg_options*, aapdhg_server_t* out) {
  if (out) *out = nullptr;
  g_thread_error = "server not available in this build";
  return AAPDHG_E_STATE;
}
aapdhg_status aapdhg_server_submit(aapdhg_server_t, int32_t, int32_t, int64_t, const int64_t*, const int32_t*,
                                   const double*, const double*, const double*, const double*, const double*,
                                   const uint8_t*, uint64_t*) {
  g_thread_error = "server not available in this build";
  return AAPDHG_E_STATE;
}
aapdhg_status aapdhg_server_poll(aapdhg_server_t, uint64_t, aapdhg_info*, double*, double*, double*, double*) {
  g_thread_error = "server not available in this build";
  return AAPDHG_E_STATE;
}
aapdhg_status aapdhg_server_stats(aapdhg_server_t, int64_t*) {
  g_thread_error = "server not available in this build";
  return AAPDHG_E_STATE;
}
aapdhg_status aapdhg_server_stop(aapdhg_server_t) { return AAPDHG_OK; }

}  // extern "C"
