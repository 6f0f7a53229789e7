// Library version and thread-local error reporting.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "common.h"

namespace vbm {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

vbm_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return VBM_OK;
  set_error("%s: HIP error %d (%s)", what, static_cast<int>(e), hipGetErrorString(e));
  return VBM_ERR_HIP;
}

}  // namespace vbm

extern "C" const char* vbm_version(void) { return "vbm-mi355x 0.1.0 (gfx950)"; }

extern "C" const char* vbm_last_error(void) { return vbm::g_last_error.c_str(); }
