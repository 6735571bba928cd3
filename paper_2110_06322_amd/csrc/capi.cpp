// Error plumbing and version queries of the C ABI.
#include <hip/hip_runtime_api.h>

#include <string>

#include "internal.h"

namespace cpm {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

[[noreturn]] void fail(cpm_status code, const std::string& msg) { throw Error{code, msg}; }

}  // namespace cpm

const char* cpm_last_error(void) { return cpm::g_last_error.c_str(); }

int32_t cpm_version(void) { return CPM_VERSION; }

int32_t cpm_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

int64_t cpm_abi_sizeof(int32_t which) {
  switch (which) {
    case 0: return (int64_t)sizeof(cpm_solve_opts);
    case 1: return (int64_t)sizeof(cpm_solve_stats);
    case 2: return (int64_t)sizeof(cpm_precond_opts);
    case 3: return (int64_t)sizeof(cpm_tune_result);
    case 4: return (int64_t)sizeof(cpm_imex_opts);
    case 5: return (int64_t)sizeof(cpm_band_info);
    case 6: return (int64_t)sizeof(cpm_operator_opts);
    case 7: return (int64_t)sizeof(cpm_operator_info);
    default: return -1;
  }
}
