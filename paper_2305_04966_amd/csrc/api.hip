// Error reporting and version of the txs C ABI.
#include <cstring>

#include "txs_common.h"

namespace txs {
namespace {
thread_local char g_error[512] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_error, sizeof(g_error), fmt, ap);
  va_end(ap);
}

void clear_error() { g_error[0] = '\0'; }

txs_status launch_status(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("%s: HIP error %d (%s)", what, (int)e, hipGetErrorString(e));
    return TXS_EHIP;
  }
  return TXS_OK;
}

}  // namespace txs

extern "C" const char* txs_last_error(void) { return txs::g_error; }

extern "C" int32_t txs_abi_version(void) { return TXS_ABI_VERSION; }
