// Error reporting and version of the LABFM C ABI.
#include <cstdarg>
#include <cstdio>

#include "../../include/labfm.h"

namespace labfm {

namespace {
thread_local char g_error[512] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_error, sizeof(g_error), fmt, ap);
  va_end(ap);
}

void clear_error() { g_error[0] = '\0'; }

}  // namespace labfm

extern "C" const char* labfm_last_error(void) { return labfm::g_error; }

extern "C" const char* labfm_version(void) { return "labfm-mi355x 0.2.0 (gfx950)"; }

extern "C" int64_t labfm_w32_stride(int64_t nnz) { return nnz <= 0 ? 0 : (nnz + 31) / 32 * 32; }
