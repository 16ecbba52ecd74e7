// Status strings, per-thread HIP error record and version of librsv.
#include <hip/hip_runtime.h>

#include "rsv.h"
#include "rsv_internal.hpp"

namespace rsv {
namespace {
thread_local int g_last_hip_error = 0;
}
void set_hip_error(hipError_t e) { g_last_hip_error = static_cast<int>(e); }
}  // namespace rsv

extern "C" const char* rsv_status_string(int status) {
  switch (status) {
    case RSV_OK: return "ok";
    case RSV_E_NULL: return "a required pointer is NULL";
    case RSV_E_SHAPE: return "size out of range (image/volume shape, pitch or D)";
    case RSV_E_PARAM: return "parameter out of range (radius, gamma, sigma_min, threshold)";
    case RSV_E_DTYPE: return "unsupported image element type";
    case RSV_E_ALIGN: return "pointer not aligned to its element size";
    case RSV_E_HIP: return "HIP runtime call failed (see rsv_last_hip_error)";
    case RSV_E_NOMEM: return "device allocation failed";
    default: return "unknown status";
  }
}

extern "C" int rsv_last_hip_error(void) { return rsv::g_last_hip_error; }

extern "C" int rsv_version(void) { return 100; }
